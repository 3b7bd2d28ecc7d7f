// Host side of the C ABI declared in include/fastnerf.h: argument checks,
// cache lifetime, per-stream launch state and kernel dispatch.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <atomic>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "fastnerf.h"
#include "fastnerf_internal.h"
#include "fastnerf_kernels.h"

using namespace fnr;

// ------------------------------------------------------------------ errors

namespace fnr {

static thread_local std::string g_err;

fastnerf_status fail(fastnerf_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

fastnerf_status hip_fail(hipError_t e, const char *what) {
  return fail(e == hipErrorOutOfMemory ? FASTNERF_ENOMEM : FASTNERF_EDEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

}  // namespace fnr

#define HIP_TRY(call)                                 \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

extern "C" const char *fastnerf_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ helpers

namespace fnr {

static int ilog2(uint64_t v) {
  int r = 0;
  while ((1ull << r) < v) ++r;
  return r;
}

bool is_device_ptr(const void *p) {
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

static bool finite_all(const float *v, int n) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(v[i])) return false;
  return true;
}

// Per (device, stream) launch state: the self-resetting tile-queue counters and
// a ring of staging slots for batched view descriptors. A batch writes its
// descriptors into the next slot's pinned buffer and copies them to the slot's
// device buffer on the stream; the host waits only if that slot's previous copy
// (kStageRing batches back) has not run yet, so batches enqueue without waiting
// for earlier launches. Allocated once per stream.
constexpr int kStageRing = 8;

struct StageSlot {
  DevView *views = nullptr;       // device
  DevView *views_host = nullptr;  // pinned
  int cap = 0;
  hipEvent_t copied = nullptr;    // recorded after the slot's last descriptor copy
};

struct StreamState {
  unsigned *counter = nullptr;
  StageSlot slot[kStageRing];
  int next = 0;                   // ring position of the next batch
  std::mutex mu;                  // held while a batch takes and fills its slot
};

static std::mutex g_streams_mu;
static std::map<std::pair<int, hipStream_t>, StreamState *> g_streams;

fastnerf_status stream_state(hipStream_t s, StreamState **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_streams_mu);
  auto key = std::make_pair(dev, s);
  auto it = g_streams.find(key);
  if (it != g_streams.end()) {
    *out = it->second;
    return FASTNERF_OK;
  }
  StreamState *st = new StreamState();
  hipError_t e = hipMalloc(&st->counter, kQueueCounters * sizeof(unsigned));
  if (e == hipSuccess) e = hipMemset(st->counter, 0, kQueueCounters * sizeof(unsigned));
  for (int q = 0; q < kStageRing && e == hipSuccess; ++q)
    e = hipEventCreateWithFlags(&st->slot[q].copied, hipEventDisableTiming);
  if (e != hipSuccess) {
    delete st;
    return hip_fail(e, "stream state");
  }
  g_streams[key] = st;
  *out = st;
  return FASTNERF_OK;
}

// The staging slot of the next batch on this stream, holding at least n
// descriptors; waits for the slot's previous copy (kStageRing batches back).
fastnerf_status stream_slot(StreamState *st, int n, StageSlot **out) {
  StageSlot *sl = &st->slot[st->next];
  st->next = (st->next + 1) % kStageRing;
  HIP_TRY(hipEventSynchronize(sl->copied));
  if (n > sl->cap) {
    if (sl->views) HIP_TRY(hipFree(sl->views));
    if (sl->views_host) HIP_TRY(hipHostFree(sl->views_host));
    sl->views = nullptr;
    sl->views_host = nullptr;
    sl->cap = 0;
    int cap = n < 64 ? 64 : n;
    HIP_TRY(hipMalloc(&sl->views, sizeof(DevView) * cap));
    HIP_TRY(hipHostMalloc(&sl->views_host, sizeof(DevView) * cap, hipHostMallocDefault));
    sl->cap = cap;
  }
  *out = sl;
  return FASTNERF_OK;
}

// Launch shape of the render kernel for a cache: a persistent grid of as many
// 256-thread blocks as are resident at once, capped by the work.
struct LaunchPlan {
  int block, grid;
};

// 32-bit words of a cache's occupancy bitgrid (one word without a bitgrid).
int occ_words_of(const fastnerf_cache_s *c) {
  return c->desc.brick > 0 ? (int)(((uint64_t)c->nbo * c->nbo * c->nbo + 31) / 32) : 1;
}

LaunchPlan launch_plan(const fastnerf_cache_s *c, int total_tiles, bool vox, int sched,
                       int64_t fill_px) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, int> plans;  // (device, variant) -> resident blocks
  int dev = 0;
  (void)hipGetDevice(&dev);
  const bool lin = c->desc.pos_interp == FASTNERF_LINEAR;
  const bool sparse = c->desc.sparse && !vox;
  if (vox) sched = kSchedTiles;
  const int occ_words = occ_words_of(c);
  const int block = vox ? kBlock
                        : render_block((int)c->desc.storage, lin, c->desc.D, sparse, sched,
                                       occ_words);
  const int variant = (int)c->desc.storage * 256 + sched * 64 + (lin ? 32 : 0) +
                      (vox ? 16 : 0) + (sparse ? 8 : 0) + (block != kBlock ? 4 : 0) +
                      (c->desc.D <= 4 ? 0 : c->desc.D <= 8 ? 1 : 2);
  int blocks;
  {
    std::lock_guard<std::mutex> g(mu);
    auto key = std::make_pair(dev, variant);
    auto it = plans.find(key);
    if (it == plans.end()) {
      int cus = 0;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          cus < 1)
        cus = 1;
      const int per_cu = vox ? render_vox_occupancy((int)c->desc.storage, c->desc.D)
                             : render_occupancy((int)c->desc.storage, lin, c->desc.D, sparse,
                                                sched, occ_words);
      it = plans.emplace(key, cus * (per_cu < 1 ? 1 : per_cu)).first;
    }
    blocks = it->second;
  }
  LaunchPlan p;
  p.block = block;
  const int wpb = p.block / kWave;
  int need = (total_tiles + wpb - 1) / wpb;
  // enough threads that the background pass writes about 64 pixels each
  const int64_t fill_blocks = (fill_px + 64 * (int64_t)p.block - 1) / (64 * (int64_t)p.block);
  if (fill_blocks > need) need = (int)std::min<int64_t>(fill_blocks, (int64_t)blocks);
  p.grid = need < blocks ? (need < 1 ? 1 : need) : blocks;
  return p;
}

// View descriptor from K and c2w; R K^-1 is formed and kept in double.
void make_view(const fastnerf_cache_s *c, const float K[9], const float c2w[12], int H, int W,
               float near_, float far_, float *out, int tile_begin, DevView *v) {
  const double a = K[0], b = K[1], cc = K[2], d = K[3], e = K[4], f = K[5], g = K[6], h = K[7],
               i = K[8];
  const double c00 = e * i - f * h, c01 = -(d * i - f * g), c02 = d * h - e * g;
  const double det = a * c00 + b * c01 + cc * c02;
  const double Ki[9] = {c00 / det, -(b * i - cc * h) / det, (b * f - cc * e) / det,
                        c01 / det, (a * i - cc * g) / det,  -(a * f - cc * d) / det,
                        c02 / det, -(a * h - b * g) / det,  (a * e - b * d) / det};
  for (int r = 0; r < 3; ++r)
    for (int col = 0; col < 3; ++col) {
      double s = 0.0;
      for (int q = 0; q < 3; ++q) s += (double)c2w[4 * r + q] * Ki[3 * q + col];
      v->M[3 * r + col] = s;
    }
  for (int r = 0; r < 3; ++r) v->o[r] = c2w[4 * r + 3];
  (void)c;
  v->near_ = near_;
  v->far_ = far_;
  v->H = H;
  v->W = W;
  v->cx0 = v->cy0 = 0;
  v->cx1 = W;
  v->cy1 = H;
  v->tile_begin = tile_begin;
  v->tile_offset = 0;
  v->scene = 0;
  v->out = out;
}

// Narrows view v's render rectangle to the pixels whose rays can meet the
// box: with every box corner in front of the camera, the box projects into
// the convex hull of its corners' projections, so a pixel whose centre ray
// meets the box lies in the corners' bounding rectangle (widened by a pixel,
// its edges rounded out to multiples of 8 and clipped to the image). A ray
// outside it takes no sample in the box, and its pixel is the background
// however it is sampled. Left whole when a corner is not in front.
void cull_view(const fastnerf_cache_s *c, const float K[9], const float c2w[12], DevView *v) {
  double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
  for (int q = 0; q < 8; ++q) {
    double X[3], Xc[3];
    for (int a = 0; a < 3; ++a)
      X[a] = ((q >> a) & 1) ? (double)c->desc.bbox_max[a] : (double)c->desc.bbox_min[a];
    // camera coordinates: R^T (X - o), R = the first three columns of c2w
    for (int col = 0; col < 3; ++col) {
      double s = 0.0;
      for (int r = 0; r < 3; ++r) s += (double)c2w[4 * r + col] * (X[r] - (double)c2w[4 * r + 3]);
      Xc[col] = s;
    }
    double u[3];
    for (int r = 0; r < 3; ++r)
      u[r] = (double)K[3 * r] * Xc[0] + (double)K[3 * r + 1] * Xc[1] + (double)K[3 * r + 2] * Xc[2];
    if (!(Xc[2] > 1e-9) || !(u[2] > 1e-9)) return;  // not in front: the whole image
    for (int a = 0; a < 2; ++a) {
      const double p = u[a] / u[2];
      if (!std::isfinite(p)) return;
      lo[a] = std::min(lo[a], p);
      hi[a] = std::max(hi[a], p);
    }
  }
  const int lim[2] = {v->W, v->H};
  int r0[2], r1[2];
  for (int a = 0; a < 2; ++a) {
    const double l = std::floor(lo[a]) - 1.0, h = std::ceil(hi[a]) + 1.0;
    const double lc = std::min(std::max(l, 0.0), (double)lim[a]);
    const double hc = std::min(std::max(h, 0.0), (double)lim[a]);
    r0[a] = ((int)lc) & ~7;
    r1[a] = std::min(lim[a], (((int)hc) + 7) & ~7);
    if (r1[a] < r0[a]) r1[a] = r0[a];
  }
  v->cx0 = r0[0];
  v->cx1 = r1[0];
  v->cy0 = r0[1];
  v->cy1 = r1[1];
}

// Tiles of edge T (8 or 4) covering view v's render rectangle.
int view_tiles(const DevView &v, int T) {
  if (v.cx1 <= v.cx0 || v.cy1 <= v.cy0) return 0;
  return ((v.cx1 + T - 1) / T - v.cx0 / T) * ((v.cy1 + T - 1) / T - v.cy0 / T);
}

// Pixels of view v outside its render rectangle.
int64_t view_outside(const DevView &v) {
  return (int64_t)v.W * v.H - (int64_t)(v.cx1 - v.cx0) * (v.cy1 - v.cy0);
}

fastnerf_status check_view(const float *K, const float *c2w, int H, int W, float near_,
                                  float far_, const float *out) {
  if (!K || !c2w || !out) return fail(FASTNERF_EINVAL, "null K, c2w or out");
  if (H <= 0 || W <= 0 || H > 65536 || W > 65536)
    return fail(FASTNERF_EINVAL, "image size %d x %d out of range", W, H);
  if (!finite_all(K, 9) || !finite_all(c2w, 12)) return fail(FASTNERF_EINVAL, "non-finite camera");
  const double det = (double)K[0] * ((double)K[4] * K[8] - (double)K[5] * K[7]) -
                     (double)K[1] * ((double)K[3] * K[8] - (double)K[5] * K[6]) +
                     (double)K[2] * ((double)K[3] * K[7] - (double)K[4] * K[6]);
  if (det == 0.0) return fail(FASTNERF_EINVAL, "singular intrinsics");
  if (!isfinite(near_) || !isfinite(far_) || !(near_ < far_))
    return fail(FASTNERF_EINVAL, "need finite near < far");
  return FASTNERF_OK;
}

DevCache dev_cache(const fastnerf_cache_s *c) {
  DevCache d;
  memset(&d, 0, sizeof d);
  const fastnerf_cache_desc &ds = c->desc;
  d.rec = c->rec;
  d.beta = c->beta;
  d.occ = c->occ;
  d.dist = c->dist;
  d.scales = c->scales;
  d.slot = ds.sparse ? c->slot : nullptr;
  d.rank = ds.sparse ? c->rank : nullptr;
  d.k = ds.k;
  d.D = ds.D;
  d.l = ds.l;
  d.bq = (ds.D + 3) / 4;
  d.nbl = c->nbl;
  d.nbo = c->desc.brick > 0 ? c->nbo : 1;
  d.occ_words = occ_words_of(c);
  d.oshift = c->desc.brick > 0 ? c->oshift : 30;
  d.nbd = c->desc.brick > 0 ? c->nbd : 1;
  d.dshift = c->desc.brick > 0 ? c->dshift : 30;
  d.rec_shift = c->rec_shift;
  d.nchunk = c->nchunk;
  d.kf = (float)ds.k;
  for (int a = 0; a < 3; ++a) {
    d.bmin[a] = ds.bbox_min[a];
    d.bmax[a] = ds.bbox_max[a];
    d.inv_h[a] = (float)((double)ds.k / ((double)ds.bbox_max[a] - (double)ds.bbox_min[a]));
    d.bg[a] = ds.background[a];
  }
  d.th_scale = (float)(ds.l / M_PI);
  d.ph_scale = (float)(ds.l / (2.0 * M_PI));
  d.in_box = ds.sample_mode == FASTNERF_SAMPLES_IN_BOX;
  d.dir_linear = ds.dir_interp == FASTNERF_LINEAR;
  d.fmt = (int)ds.storage;
  return d;
}

// Voxel traversal (N = 0) needs nearest lookups and a 32-bit record index.
static fastnerf_status check_voxel_mode(const fastnerf_cache_s *c, int N) {
  if (N != 0) return FASTNERF_OK;
  if (c->desc.pos_interp != FASTNERF_NEAREST)
    return fail(FASTNERF_EINVAL, "N = 0 (voxel traversal) needs nearest position lookups");
  if (c->desc.k > 1024) return fail(FASTNERF_EINVAL, "N = 0 (voxel traversal) needs k <= 1024");
  return FASTNERF_OK;
}

fastnerf_status check_render_params(int N, float eps) {
  if (N < 0 || N > 4096) return fail(FASTNERF_EINVAL, "N = %d outside [0, 4096]", N);
  if (!(eps >= 0.0f && eps < 1.0f)) return fail(FASTNERF_EINVAL, "eps outside [0, 1)");
  return FASTNERF_OK;
}

float eps_limit(float eps) { return eps > 0.0f ? (float)log(1.0 / (double)eps) : INFINITY; }

// Scheduling of fixed-N render launches (fastnerf_set_schedule).
static std::atomic<int> g_schedule{FASTNERF_SCHEDULE_AUTO};

// Launches of at most this many tiles (about two 800x800 views) cannot fill
// the chip with the throughput kernels' waves, and are bound by the dependency
// chains of their heaviest rays: AUTO gives them the wide kernel.
constexpr int kWideMaxTiles = 20000;
#ifndef FNR_AUTO_SPLIT
#define FNR_AUTO_SPLIT 1
#endif
constexpr bool kAutoSplit = FNR_AUTO_SPLIT != 0;
// Views per interleaved group of a batch of one view size (0: none).
#ifndef FNR_INTERLEAVE
#define FNR_INTERLEAVE 8
#endif
constexpr int kInterleave = FNR_INTERLEAVE;


// Whether a launch can take split rays: a single view (no view array) of a
// dense cache with nearest lookups and at most 8 components.
bool split_ok(const fastnerf_cache_s *c, const RenderArgs &a) {
  return !a.views && !c->desc.sparse && c->desc.pos_interp == FASTNERF_NEAREST &&
         c->desc.D <= 8;
}

// The schedule of a launch (kSched*): AUTO takes split rays for a small
// single-view launch that can take them, the wide kernel for other small
// launches and tiles otherwise (measured on the paper-scale orbit, the refill
// schedule was slower: its lanes hold rays of different tiles, so the lanes'
// occupied samples per window are less alike and the gather rounds of a
// window, the most over the wave's lanes, grow). SPLIT asked for a launch
// that cannot take it runs WIDE.
int launch_schedule(const fastnerf_cache_s *c, const RenderArgs &a, int total_tiles) {
  if (a.vox) return kSchedTiles;
  switch (g_schedule.load(std::memory_order_relaxed)) {
    case FASTNERF_SCHEDULE_TILES: return kSchedTiles;
    case FASTNERF_SCHEDULE_REFILL: return kSchedRefill;
    case FASTNERF_SCHEDULE_WIDE: return kSchedWide;
    case FASTNERF_SCHEDULE_SPLIT: return split_ok(c, a) ? kSchedSplit : kSchedWide;
    default: break;
  }
  if (total_tiles > kWideMaxTiles) return kSchedTiles;
  return (kAutoSplit && split_ok(c, a)) ? kSchedSplit : kSchedWide;
}

fastnerf_status enqueue_render(fastnerf_cache_s *c, const RenderArgs &a0, int total_tiles,
                               unsigned *counter, hipStream_t s) {
  RenderArgs a = a0;
  a.sched = launch_schedule(c, a, total_tiles);
  // split rays take 4x4-pixel tiles
  if (a.sched == kSchedSplit) total_tiles = view_tiles(a.v0, 4);
  if (!a.views) a.fill_px = view_outside(a.v0);
  const LaunchPlan p = launch_plan(c, total_tiles, a.vox != 0, a.sched, a.fill_px);
  a.counter = counter;
  a.nwaves = (unsigned)p.grid * (p.block / kWave);
  a.total_tiles = total_tiles;
  hipError_t e = a.vox ? launch_render_vox((int)c->desc.storage, a, p.grid, s)
                       : launch_render((int)c->desc.storage,
                                       c->desc.pos_interp == FASTNERF_LINEAR, a, p.grid, s);
  if (e != hipSuccess) return hip_fail(e, "render launch");
  HIP_TRY(hipEventRecord(c->last_use, s));
  return FASTNERF_OK;
}

}  // namespace fnr

// ------------------------------------------------------------------ caches

static fastnerf_status validate_desc(const fastnerf_cache_desc *d) {
  if (!d) return fail(FASTNERF_EINVAL, "null descriptor");
  if (d->k < 1 || d->k > 4096) return fail(FASTNERF_EINVAL, "k = %d outside [1, 4096]", d->k);
  if (d->D < 1 || d->D > 16) return fail(FASTNERF_EINVAL, "D = %d outside [1, 16]", d->D);
  if (d->l < 1 || d->l > 4096) return fail(FASTNERF_EINVAL, "l = %d outside [1, 4096]", d->l);
  if ((unsigned)d->storage > 3u) return fail(FASTNERF_EINVAL, "unknown storage format");
  if ((unsigned)d->pos_interp > 1u || (unsigned)d->dir_interp > 1u)
    return fail(FASTNERF_EINVAL, "unknown interpolation mode");
  if ((unsigned)d->sample_mode > 1u) return fail(FASTNERF_EINVAL, "unknown sample mode");
  if (d->brick < 0 || (d->brick > 0 && ((d->brick & (d->brick - 1)) || d->k % d->brick)))
    return fail(FASTNERF_EINVAL, "brick %d must be 0 or a power of two dividing k = %d",
                d->brick, d->k);
  if (d->brick > 0 && d->k / d->brick > 1024)
    return fail(FASTNERF_EINVAL, "k / brick = %d exceeds 1024 bricks per axis",
                d->k / d->brick);
  for (int a = 0; a < 3; ++a)
    if (!isfinite(d->bbox_min[a]) || !isfinite(d->bbox_max[a]) ||
        !(d->bbox_min[a] < d->bbox_max[a]) || !isfinite(d->background[a]))
      return fail(FASTNERF_EINVAL, "bad bounding box or background");
  if ((unsigned)d->sparse > 1u) return fail(FASTNERF_EINVAL, "sparse must be 0 or 1");
  if (d->sparse && (d->pos_interp != FASTNERF_NEAREST || d->brick != 8 || d->k % 8))
    return fail(FASTNERF_EINVAL, "a brick-sparse cache needs nearest lookups, brick = 8 and "
                                 "k %% 8 == 0");
  return FASTNERF_OK;
}

extern "C" fastnerf_status fastnerf_cache_create_empty(const fastnerf_cache_desc *desc,
                                                       const float *beta, hipStream_t stream,
                                                       fastnerf_cache *out) {
  fastnerf_status st = validate_desc(desc);
  if (st != FASTNERF_OK) return st;
  if (!beta || !out) return fail(FASTNERF_EINVAL, "null beta or out");
  *out = nullptr;
  fastnerf_cache_s *c = new (std::nothrow) fastnerf_cache_s();
  if (!c) return fail(FASTNERF_ENOMEM, "host allocation");
  c->desc = *desc;
  const int sz = desc->storage == FASTNERF_F32 ? 4 : desc->storage == FASTNERF_FP8_E4M3 ? 1 : 2;
  c->payload = (1 + 3 * desc->D) * sz;
  // records hold the chunks that the kernels for this component count load
  // (zero past the payload); the stride is the next power of two
  c->nchunk = ((1 + 3 * maxd_class(desc->D)) * sz + 15) / 16;
  int stride = 16;
  while (stride < c->nchunk * 16) stride <<= 1;
  c->stride = stride;
  c->rec_shift = ilog2((uint64_t)stride);
  c->nbl = (desc->k + 7) / 8;
  if (desc->brick > 0) {
    c->oshift = ilog2((uint64_t)desc->brick);
    c->nbo = desc->k / desc->brick;
    // the distance field keeps 8^3 bricks under a finer bitgrid (one byte per
    // brick of a 4^3 or 2^3 grid would no longer stay in the L2 at k = 768)
    const int db = desc->brick < 8 && desc->k % 8 == 0 ? 8 : desc->brick;
    c->dshift = ilog2((uint64_t)db);
    c->nbd = desc->k / db;
  } else {
    c->oshift = 0;
    c->nbo = 0;
    c->dshift = 0;
    c->nbd = 0;
  }
  const uint64_t nlb = (uint64_t)c->nbl * c->nbl * c->nbl;
  // a brick-sparse cache allocates its records once the stored bricks are known
  const uint64_t rec_bytes = desc->sparse ? 0 : nlb * 512ull * (uint64_t)stride;
  const int dp = (desc->D + 3) / 4 * 4;  // direction-cache row, padded to 16 bytes
  const uint64_t beta_bytes = (uint64_t)desc->l * desc->l * dp * sizeof(float);
  const uint64_t nbits = (uint64_t)c->nbo * c->nbo * c->nbo;
  // one word more than the bitgrid, rounded up to 16 bytes (the LDS-staged
  // kernels copy whole 16-byte chunks)
  const uint64_t occ_bytes = ((nbits + 31) / 32 + 1 + 3) / 4 * 16;
  const uint64_t ndist = (uint64_t)c->nbd * c->nbd * c->nbd;
  const uint64_t dist_bytes = ndist > 0 ? ndist : 1;
  const int nch = 1 + 3 * desc->D;
  const uint64_t nwords = occ_bytes / 4;
  const uint64_t sparse_bytes = desc->sparse ? nlb * 4 + nwords * 4 : 0;  // slot, rank
  hipError_t e = hipSuccess;
  if (rec_bytes) e = hipMalloc(&c->rec, rec_bytes);
  if (e == hipSuccess && desc->sparse) e = hipMalloc(&c->bflag, nlb * 4);
  if (e == hipSuccess && desc->sparse) e = hipMalloc(&c->slot, nlb * 4);
  if (e == hipSuccess && desc->sparse) e = hipMalloc(&c->rank, nwords * 4);
  if (e == hipSuccess && desc->sparse) e = hipMemsetAsync(c->bflag, 0, nlb * 4, stream);
  if (e == hipSuccess) e = hipMalloc(&c->beta, beta_bytes);
  if (e == hipSuccess) e = hipMalloc(&c->occ, occ_bytes);
  if (e == hipSuccess) e = hipMalloc(&c->dist, dist_bytes);
  if (e == hipSuccess) e = hipMalloc(&c->scales, sizeof(float) * kMaxCh);
  if (e == hipSuccess) e = hipMalloc(&c->amax, sizeof(unsigned) * nch);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->last_use, hipEventDisableTiming);
  if (e == hipSuccess && rec_bytes) e = hipMemsetAsync(c->rec, 0, rec_bytes, stream);
  // without a bitgrid the kernels read one all-ones word and one zero distance
  if (e == hipSuccess) e = hipMemsetAsync(c->occ, desc->brick > 0 ? 0 : 0xFF, occ_bytes, stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->dist, 0, dist_bytes, stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->amax, 0, sizeof(unsigned) * nch, stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->beta, 0, beta_bytes, stream);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(c->beta, dp * sizeof(float), beta, desc->D * sizeof(float),
                         desc->D * sizeof(float), (size_t)desc->l * desc->l, hipMemcpyDefault,
                         stream);
  std::vector<float> ones(kMaxCh, 1.0f);  // FP8 overwrites the first 1 + 3D
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->scales, ones.data(), sizeof(float) * kMaxCh, hipMemcpyHostToDevice,
                       stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (desc->storage != FASTNERF_FP8_E4M3) c->scales_ready = true;
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    fastnerf_status r = hip_fail(e, "cache allocation");
    fastnerf_cache_destroy(c);
    return r;
  }
  c->resident =
      rec_bytes + sparse_bytes + beta_bytes + occ_bytes + dist_bytes + sizeof(float) * kMaxCh;
  c->occ_bytes = occ_bytes;
  (void)hipGetDevice(&c->device);
  *out = c;
  return FASTNERF_OK;
}

// Runs fn(sigma_dev, u_dev, z0, nz) over the slab, staging host input through
// device memory in chunks of layers.
template <class Fn>
static fastnerf_status for_device_slab(fastnerf_cache_s *c, int z0, int nz, const float *sigma,
                                       const float *u, hipStream_t s, Fn fn) {
  const int k = c->desc.k, n3 = 3 * c->desc.D;
  const bool dev = is_device_ptr(sigma);
  if (dev != is_device_ptr(u)) return fail(FASTNERF_EINVAL, "sigma and u must both be host or device");
  if (dev) return fn(sigma, u, z0, nz);
  const uint64_t layer = (uint64_t)k * k;
  int chunk = (int)((256ull << 20) / (layer * (1 + n3) * 4));
  if (chunk < 1) chunk = 1;
  if (chunk > nz) chunk = nz;
  float *ds = nullptr, *du = nullptr;
  hipError_t e = hipMalloc(&ds, layer * chunk * 4);
  if (e == hipSuccess) e = hipMalloc(&du, layer * chunk * n3 * 4);
  fastnerf_status st = FASTNERF_OK;
  for (int z = 0; e == hipSuccess && st == FASTNERF_OK && z < nz; z += chunk) {
    const int m = nz - z < chunk ? nz - z : chunk;
    e = hipMemcpyAsync(ds, sigma + (uint64_t)z * layer, layer * m * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(du, u + (uint64_t)z * layer * n3, layer * m * n3 * 4,
                         hipMemcpyHostToDevice, s);
    if (e == hipSuccess) st = fn(ds, du, z0 + z, m);
    if (e == hipSuccess && st == FASTNERF_OK) e = hipStreamSynchronize(s);
  }
  if (ds) (void)hipFree(ds);
  if (du) (void)hipFree(du);
  if (e != hipSuccess) return hip_fail(e, "slab staging");
  return st;
}

static fastnerf_status check_slab(fastnerf_cache_s *c, int z0, int nz, const float *sigma,
                                  const float *u) {
  if (!c) return fail(FASTNERF_EINVAL, "null cache");
  if (c->finalized) return fail(FASTNERF_EINVAL, "cache already finalized");
  if (!sigma || !u) return fail(FASTNERF_EINVAL, "null sigma or u");
  if (z0 < 0 || nz < 1 || z0 + nz > c->desc.k)
    return fail(FASTNERF_EINVAL, "slab [%d, %d) outside [0, %d)", z0, z0 + nz, c->desc.k);
  return FASTNERF_OK;
}

extern "C" fastnerf_status fastnerf_cache_scan_slab(fastnerf_cache c, int32_t z0, int32_t nz,
                                                    const float *sigma, const float *u,
                                                    hipStream_t s) {
  fastnerf_status st = check_slab(c, z0, nz, sigma, u);
  if (st != FASTNERF_OK) return st;
  const bool fp8 = c->desc.storage == FASTNERF_FP8_E4M3, sparse = c->desc.sparse != 0;
  if (!fp8 && !sparse) return FASTNERF_OK;
  if ((fp8 && c->scales_ready) || (sparse && c->sparse_ready))
    return fail(FASTNERF_EINVAL, "scan after the first upload");
  if (sparse) c->scanned = true;
  return for_device_slab(c, z0, nz, sigma, u, s,
                         [&](const float *ds, const float *du, int zz, int m) -> fastnerf_status {
                           hipError_t e = hipSuccess;
                           if (fp8)
                             e = launch_absmax(ds, du, (int64_t)m * c->desc.k * c->desc.k,
                                               c->desc.D, c->amax, s);
                           if (e == hipSuccess && sparse)
                             e = launch_brick_flags(ds, zz, m, c->desc.k, c->nbl, c->bflag, s);
                           return e == hipSuccess ? FASTNERF_OK : hip_fail(e, "slab scan");
                         });
}

// Brick-sparse caches, at the first upload: from the brick flags of the scan,
// the bitgrid (bit = brick stored), the set bits before each bitgrid word, the
// stored slot of every brick (1 + its rank; 0 = the all-zero brick) and the
// records of the stored bricks, zeroed.
static fastnerf_status build_sparse_layout(fastnerf_cache_s *c, hipStream_t s) {
  if (!c->scanned) return fail(FASTNERF_EINVAL, "a brick-sparse cache needs scan_slab first");
  const uint64_t nlb = (uint64_t)c->nbl * c->nbl * c->nbl;
  const uint64_t nwords = c->occ_bytes / 4;
  std::vector<uint32_t> flags(nlb), words(nwords, 0u), rank(nwords, 0u);
  std::vector<int32_t> slot(nlb, 0);
  HIP_TRY(hipMemcpyAsync(flags.data(), c->bflag, nlb * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  uint64_t n = 0;
  for (uint64_t b = 0; b < nlb; ++b) {
    if ((b & 31) == 0) rank[b >> 5] = (uint32_t)n;
    if (flags[b]) {
      words[b >> 5] |= 1u << (b & 31);
      slot[b] = (int32_t)(++n);
    }
  }
  for (uint64_t w = (nlb + 31) / 32; w < nwords; ++w) rank[w] = (uint32_t)n;
  const uint64_t rec_bytes = (n + 1) * 512ull * (uint64_t)c->stride;
  hipError_t e = hipMalloc(&c->rec, rec_bytes);
  if (e == hipSuccess) e = hipMemsetAsync(c->rec, 0, rec_bytes, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->occ, words.data(), nwords * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->rank, rank.data(), nwords * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->slot, slot.data(), nlb * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "sparse layout");
  (void)hipFree(c->bflag);
  c->bflag = nullptr;
  c->nstored = n;
  c->resident += rec_bytes;
  c->sparse_ready = true;
  return FASTNERF_OK;
}

extern "C" fastnerf_status fastnerf_cache_upload_slab(fastnerf_cache c, int32_t z0, int32_t nz,
                                                      const float *sigma, const float *u,
                                                      hipStream_t s) {
  fastnerf_status st = check_slab(c, z0, nz, sigma, u);
  if (st != FASTNERF_OK) return st;
  if (!c->scales_ready) {
    hipError_t e = launch_make_scales(c->amax, 1 + 3 * c->desc.D, c->scales, s);
    if (e != hipSuccess) return hip_fail(e, "scales");
    c->scales_ready = true;
  }
  if (c->desc.sparse && !c->sparse_ready) {
    st = build_sparse_layout(c, s);
    if (st != FASTNERF_OK) return st;
  }
  const DevCache dc = dev_cache(c);
  return for_device_slab(c, z0, nz, sigma, u, s,
                         [&](const float *ds, const float *du, int zz, int m) -> fastnerf_status {
                           hipError_t e = launch_pack((int)c->desc.storage, ds, du, zz, m, dc, s);
                           return e == hipSuccess ? FASTNERF_OK : hip_fail(e, "pack");
                         });
}

extern "C" fastnerf_status fastnerf_cache_finalize(fastnerf_cache c, hipStream_t s) {
  if (!c) return fail(FASTNERF_EINVAL, "null cache");
  if (c->finalized) return fail(FASTNERF_EINVAL, "cache already finalized");
  if (!c->scales_ready) return fail(FASTNERF_EINVAL, "no slab was uploaded");
  if (c->desc.brick > 0) {
    const DevCache dc = dev_cache(c);
    hipError_t e = hipSuccess;
    if (!c->desc.sparse)  // a brick-sparse bitgrid is the stored-brick set
      e = launch_occupancy((int)c->desc.storage, dc,
                           c->desc.pos_interp == FASTNERF_LINEAR ? 1 : 0, c->occ, s);
    if (e != hipSuccess) return hip_fail(e, "occupancy");
    const uint64_t nbr = (uint64_t)c->nbd * c->nbd * c->nbd;
    uint8_t *tmp = nullptr;
    e = hipMalloc(&tmp, nbr);
    if (e != hipSuccess) return hip_fail(e, "distance scratch");
    e = launch_distance(dc, c->occ, c->dist, tmp, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "distance field");
  }
  HIP_TRY(hipStreamSynchronize(s));
  c->finalized = true;
  return FASTNERF_OK;
}

extern "C" fastnerf_status fastnerf_cache_create(const fastnerf_cache_desc *desc,
                                                 const float *sigma, const float *u,
                                                 const float *beta, hipStream_t s,
                                                 fastnerf_cache *out) {
  if (!sigma || !u) return fail(FASTNERF_EINVAL, "null sigma or u");
  if (!out) return fail(FASTNERF_EINVAL, "null out");
  fastnerf_cache c = nullptr;
  fastnerf_status st = fastnerf_cache_create_empty(desc, beta, s, &c);
  if (st != FASTNERF_OK) return st;
  st = fastnerf_cache_scan_slab(c, 0, desc->k, sigma, u, s);
  if (st == FASTNERF_OK) st = fastnerf_cache_upload_slab(c, 0, desc->k, sigma, u, s);
  if (st == FASTNERF_OK) st = fastnerf_cache_finalize(c, s);
  if (st != FASTNERF_OK) {
    std::string msg = g_err;
    fastnerf_cache_destroy(c);
    g_err = msg;
    return st;
  }
  *out = c;
  return FASTNERF_OK;
}

extern "C" fastnerf_status fastnerf_cache_bytes(fastnerf_cache c, uint64_t *resident) {
  if (!c || !resident) return fail(FASTNERF_EINVAL, "null argument");
  *resident = c->resident;
  return FASTNERF_OK;
}

extern "C" fastnerf_status fastnerf_cache_record_bytes(fastnerf_cache c, int32_t *stride,
                                                       int32_t *payload) {
  if (!c || !stride || !payload) return fail(FASTNERF_EINVAL, "null argument");
  *stride = c->stride;
  *payload = c->payload;
  return FASTNERF_OK;
}

extern "C" fastnerf_status fastnerf_cache_readback(fastnerf_cache c, float *sigma, float *u,
                                                   float *scales, hipStream_t s) {
  if (!c || !sigma || !u) return fail(FASTNERF_EINVAL, "null argument");
  if (!c->finalized) return fail(FASTNERF_EINVAL, "cache not finalized");
  if (!is_device_ptr(sigma) || !is_device_ptr(u))
    return fail(FASTNERF_EINVAL, "readback buffers must be device memory");
  hipError_t e = launch_readback((int)c->desc.storage, dev_cache(c), sigma, u, s);
  if (e != hipSuccess) return hip_fail(e, "readback");
  if (scales)
    HIP_TRY(hipMemcpyAsync(scales, c->scales, sizeof(float) * (1 + 3 * c->desc.D),
                           hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return FASTNERF_OK;
}

extern "C" fastnerf_status fastnerf_cache_occupancy(fastnerf_cache c, uint32_t *words,
                                                    int32_t *n) {
  if (!c || !n) return fail(FASTNERF_EINVAL, "null argument");
  *n = c->nbo;
  if (c->desc.brick == 0 || !words) return FASTNERF_OK;
  const uint64_t nbits = (uint64_t)c->nbo * c->nbo * c->nbo;
  HIP_TRY(hipMemcpy(words, c->occ, (nbits + 31) / 32 * 4, hipMemcpyDeviceToHost));
  return FASTNERF_OK;
}

extern "C" fastnerf_status fastnerf_cache_skip_distance(fastnerf_cache c, uint8_t *dist,
                                                        int32_t *n) {
  if (!c || !n) return fail(FASTNERF_EINVAL, "null argument");
  if (!c->finalized) return fail(FASTNERF_EINVAL, "cache not finalized");
  *n = c->desc.brick > 0 ? c->nbd : 0;
  if (c->desc.brick == 0 || !dist) return FASTNERF_OK;
  const uint64_t nbr = (uint64_t)c->nbd * c->nbd * c->nbd;
  HIP_TRY(hipMemcpy(dist, c->dist, nbr, hipMemcpyDeviceToHost));
  return FASTNERF_OK;
}

extern "C" fastnerf_status fastnerf_cache_destroy(fastnerf_cache c) {
  if (!c) return fail(FASTNERF_EINVAL, "null cache");
  if (c->last_use) {
    (void)hipEventSynchronize(c->last_use);
    (void)hipEventDestroy(c->last_use);
  }
  if (c->rec) (void)hipFree(c->rec);
  if (c->beta) (void)hipFree(c->beta);
  if (c->occ) (void)hipFree(c->occ);
  if (c->dist) (void)hipFree(c->dist);
  if (c->scales) (void)hipFree(c->scales);
  if (c->amax) (void)hipFree(c->amax);
  if (c->bflag) (void)hipFree(c->bflag);
  if (c->slot) (void)hipFree(c->slot);
  if (c->rank) (void)hipFree(c->rank);
  delete c;
  return FASTNERF_OK;
}

// ------------------------------------------------------------------ rendering

extern "C" fastnerf_status fastnerf_render(fastnerf_cache c, const float K[9],
                                           const float c2w[12], int32_t H, int32_t W, float near_,
                                           float far_, int32_t N, float eps, float *out,
                                           hipStream_t s) {
  if (!c) return fail(FASTNERF_EINVAL, "null cache");
  if (!c->finalized) return fail(FASTNERF_EINVAL, "cache not finalized");
  fastnerf_status st = check_view(K, c2w, H, W, near_, far_, out);
  if (st == FASTNERF_OK) st = check_render_params(N, eps);
  if (st == FASTNERF_OK) st = check_voxel_mode(c, N);
  if (st != FASTNERF_OK) return st;
  StreamState *ss = nullptr;
  st = stream_state(s, &ss);
  if (st != FASTNERF_OK) return st;
  RenderArgs a;
  memset(&a, 0, sizeof a);
  a.c = dev_cache(c);
  make_view(c, K, c2w, H, W, near_, far_, out, 0, &a.v0);
  cull_view(c, K, c2w, &a.v0);
  a.v0.N = N;
  a.v0.lim = eps_limit(eps);
  a.views = nullptr;
  a.nviews = 1;
  a.vox = N == 0;
  return enqueue_render(c, a, view_tiles(a.v0, 8), ss->counter, s);
}

// ------------------------------------------------------------------ allocation-free render

// Tile-queue counters of fastnerf_render_noalloc: a fixed array in the
// library's own device memory, one copy per device (4 KiB), held until the
// process ends. In host code `scratch` names a host-side stand-in, not device
// memory: the kernels get the device address found once per device below.
static __device__ __align__(256) unsigned scratch[fnr::kQueueCounters];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned *g_scratch_addr[kMaxDevices];  // device address of `scratch`, per device

// Device address of the current device's `scratch`, looked up on the device's
// first call (with that device current) and kept.
static fastnerf_status scratch_address(unsigned **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FASTNERF_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "address of the render scratch counters");
    g_scratch_addr[dev] = static_cast<unsigned *>(p);
  }
  *out = g_scratch_addr[dev];
  return FASTNERF_OK;
}

extern "C" fastnerf_status fastnerf_render_noalloc(fastnerf_cache c, const float K[9],
                                                   const float c2w[12], int32_t H, int32_t W,
                                                   float near_, float far_, int32_t N, float eps,
                                                   float *out, hipStream_t s) {
  if (!c) return fail(FASTNERF_EINVAL, "null cache");
  if (!c->finalized) return fail(FASTNERF_EINVAL, "cache not finalized");
  fastnerf_status st = check_view(K, c2w, H, W, near_, far_, out);
  if (st == FASTNERF_OK) st = check_render_params(N, eps);
  if (st == FASTNERF_OK) st = check_voxel_mode(c, N);
  if (st != FASTNERF_OK) return st;
  unsigned *ctr = nullptr;
  st = scratch_address(&ctr);
  if (st != FASTNERF_OK) return st;
  // the counters start at zero on this stream whatever an earlier call left
  const hipError_t e = launch_fill_u32(ctr, kQueueCounters, 0u, s);
  if (e != hipSuccess) return hip_fail(e, "scratch counter clear");
  RenderArgs a;
  memset(&a, 0, sizeof a);
  a.c = dev_cache(c);
  make_view(c, K, c2w, H, W, near_, far_, out, 0, &a.v0);
  cull_view(c, K, c2w, &a.v0);
  a.v0.N = N;
  a.v0.lim = eps_limit(eps);
  a.views = nullptr;
  a.nviews = 1;
  a.vox = N == 0;
  return enqueue_render(c, a, view_tiles(a.v0, 8), ctr, s);
}

extern "C" fastnerf_status fastnerf_render_batch(fastnerf_cache c, int32_t nviews,
                                                 const float *K, const float *c2w,
                                                 const int32_t *H, const int32_t *W,
                                                 const float *near_, const float *far_,
                                                 int32_t N, float eps, float *const *out,
                                                 hipStream_t s) {
  if (!c) return fail(FASTNERF_EINVAL, "null cache");
  if (!c->finalized) return fail(FASTNERF_EINVAL, "cache not finalized");
  if (nviews < 1) return fail(FASTNERF_EINVAL, "nviews = %d", nviews);
  if (!K || !c2w || !H || !W || !near_ || !far_ || !out)
    return fail(FASTNERF_EINVAL, "null view array");
  fastnerf_status st = check_render_params(N, eps);
  if (st == FASTNERF_OK) st = check_voxel_mode(c, N);
  if (st != FASTNERF_OK) return st;
  int64_t total = 0;
  for (int v = 0; v < nviews; ++v) {
    st = check_view(K + 9 * v, c2w + 12 * v, H[v], W[v], near_[v], far_[v], out[v]);
    if (st != FASTNERF_OK) return fail(st, "view %d: %s", v, g_err.c_str());
    total += (int64_t)((W[v] + 7) / 8) * ((H[v] + 7) / 8);
  }
  if (total > (int64_t)0x7FFFFFFF) return fail(FASTNERF_EINVAL, "too many tiles in one batch");
  StreamState *ss = nullptr;
  StageSlot *sl = nullptr;
  st = stream_state(s, &ss);
  if (st != FASTNERF_OK) return st;
  std::lock_guard<std::mutex> guard(ss->mu);
  st = stream_slot(ss, nviews, &sl);
  if (st != FASTNERF_OK) return st;
  // the views of a batch cover their whole images (render rectangles, which
  // save the tiles that cannot see the box, measured no faster for batches);
  // views of one size are interleaved in groups, others follow one another
  bool same = kInterleave > 0 && nviews > 1;
  for (int v = 1; v < nviews && same; ++v) same = W[v] == W[0] && H[v] == H[0];
  int tb = 0;
  for (int v = 0; v < nviews; ++v) {
    make_view(c, K + 9 * v, c2w + 12 * v, H[v], W[v], near_[v], far_[v], out[v], tb,
              sl->views_host + v);
    sl->views_host[v].N = N;
    sl->views_host[v].lim = eps_limit(eps);
    tb += view_tiles(sl->views_host[v], 8);
  }
  HIP_TRY(hipMemcpyAsync(sl->views, sl->views_host, sizeof(DevView) * nviews,
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(sl->copied, s));
  RenderArgs a;
  memset(&a, 0, sizeof a);
  a.c = dev_cache(c);
  a.views = sl->views;
  a.nviews = nviews;
  a.vox = N == 0;
  a.interleave = same ? kInterleave : 0;
  a.fill_px = 0;
  for (int v = 0; v < nviews; ++v) a.fill_px += view_outside(sl->views_host[v]);
  (void)total;
  return enqueue_render(c, a, tb, ss->counter, s);
}

extern "C" fastnerf_status fastnerf_set_schedule(int32_t schedule) {
  if (schedule != FASTNERF_SCHEDULE_AUTO && schedule != FASTNERF_SCHEDULE_TILES &&
      schedule != FASTNERF_SCHEDULE_REFILL && schedule != FASTNERF_SCHEDULE_WIDE &&
      schedule != FASTNERF_SCHEDULE_SPLIT)
    return fail(FASTNERF_EINVAL, "unknown schedule %d", schedule);
  fnr::g_schedule.store(schedule, std::memory_order_relaxed);
  return FASTNERF_OK;
}

extern "C" int32_t fastnerf_get_schedule(void) {
  return fnr::g_schedule.load(std::memory_order_relaxed);
}

extern "C" fastnerf_status fastnerf_debug_lookup(fastnerf_cache c, int32_t n, const float *pts,
                                                 const float *dirs, float *sigma_u, float *beta,
                                                 hipStream_t s) {
  if (!c) return fail(FASTNERF_EINVAL, "null cache");
  if (!c->finalized) return fail(FASTNERF_EINVAL, "cache not finalized");
  if (n < 0) return fail(FASTNERF_EINVAL, "n < 0");
  if (n == 0) return FASTNERF_OK;
  if ((pts == nullptr) != (sigma_u == nullptr) || (dirs == nullptr) != (beta == nullptr))
    return fail(FASTNERF_EINVAL, "inputs and outputs must be given in pairs");
  hipError_t e = launch_lookup((int)c->desc.storage, c->desc.pos_interp == FASTNERF_LINEAR,
                               dev_cache(c), n, pts, dirs, sigma_u, beta, s);
  if (e != hipSuccess) return hip_fail(e, "lookup");
  return FASTNERF_OK;
}

extern "C" double fastnerf_model_bytes(double alpha, int64_t k, int64_t l, int32_t D,
                                       double s_sigma, double s_uvw, double s_beta) {
  const double k3 = (double)k * (double)k * (double)k;
  return alpha * (((double)D * s_uvw + s_sigma) * k3) + (double)D * s_beta * (double)l * (double)l;
}
