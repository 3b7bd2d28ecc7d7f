/*
 * fastnerf.h -- C ABI of the MI355X (gfx950) FastNeRF cached renderer.
 *
 * The library renders novel views from a factorised FastNeRF cache (Garbin et
 * al., "FastNeRF: High-Fidelity Neural Rendering at 200FPS"):
 *   - a position cache of k^3 voxels over a box V, each holding a density sigma
 *     and a deep radiance map of D components (u_i, v_i, w_i)    [Sec. 3.2 Eq. 3, Sec. 3.3]
 *   - a direction cache of l x l cells over theta in [0,pi] and phi in
 *     [0,2pi), each holding D weights beta                       [Sec. 3.2 Eq. 4, Sec. 3.3]
 * For each pixel a ray is cast, N samples are placed between the near and far
 * bounds, the colour of a sample is beta . (u, v, w)               [Sec. 3.2 Eq. 5]
 * and the samples are composited front to back with the transmittance [Sec. 3.1 Eq. 1],
 * stopping once it falls below eps                                [supplementary S3].
 *
 * Conventions (readings of the paper, which does not fix them):
 *   - Camera: pinhole intrinsics K (3x3 row-major) and camera-to-world c2w
 *     (3x4 row-major, columns right, down, forward, eye: OpenCV axes). The ray
 *     of pixel (x, y) has direction normalize(R K^-1 (x+1/2, y+1/2, 1)); row 0
 *     is the top of the image.
 *   - Samples: delta = (t1 - t0)/N, t_i = t0 + (i + 1/2) delta, where [t0, t1]
 *     is [near, far] (FASTNERF_SAMPLES_NEAR_FAR) or [near, far] clipped to the
 *     box (FASTNERF_SAMPLES_IN_BOX).
 *   - Position cache values sit at voxel centres; the nearest voxel of a point
 *     is the cell that contains it; outside the box the density is 0.
 *     Trilinear lookups clamp corner indices to the grid.
 *   - Direction: theta from +z, phi = atan2(y, x) in [0, 2pi); bilinear
 *     lookups over cell centres are periodic in phi and clamped in theta.
 *   - Compositing keeps the optical depth tau; it stops before a sample once
 *     tau > ln(1/eps) (eps = 0: never). Output RGBA: RGB = C + exp(-tau) bg,
 *     A = 1 - exp(-tau). No activation is applied to the colour.
 *   - Storage: FP32, FP16 or BF16 (round to nearest even), or OCP FP8 E4M3
 *     (round to nearest even, saturating) with one absmax scale per channel
 *     (sigma and each of the 3D radiance channels): s = absmax/448 (1 if 0),
 *     value = code * s. All arithmetic after the load is FP32.
 *
 * Errors: every call returns a fastnerf_status. Argument errors are reported
 * synchronously, before anything is enqueued; fastnerf_last_error() returns a
 * thread-local message for the last non-OK status. Render calls never
 * synchronise: a device fault surfaces at the caller's next synchronisation.
 * No C++ exception crosses the ABI.
 *
 * Memory: pointers marked "host or device" are classified with
 * hipPointerGetAttributes; the library copies what it needs and the caller
 * keeps ownership. Output buffers are caller-owned device memory.
 */
#ifndef FASTNERF_H
#define FASTNERF_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FASTNERF_OK = 0,
  FASTNERF_EINVAL = -1,    /* bad argument or call out of order */
  FASTNERF_ENOMEM = -2,    /* device or host allocation failed, or a request can never fit */
  FASTNERF_EDEVICE = -3,   /* a HIP runtime call failed */
  FASTNERF_EBUSY = -4,     /* queue full, try again */
  FASTNERF_ECANCELED = -5, /* the request was cancelled */
  FASTNERF_ESHUTDOWN = -6, /* the server is shutting down */
  FASTNERF_ETIMEDOUT = -7  /* a wait ran out of time */
} fastnerf_status;

typedef enum { FASTNERF_F32 = 0, FASTNERF_F16 = 1, FASTNERF_BF16 = 2, FASTNERF_FP8_E4M3 = 3 } fastnerf_dtype;
typedef enum { FASTNERF_NEAREST = 0, FASTNERF_LINEAR = 1 } fastnerf_interp;
typedef enum { FASTNERF_SAMPLES_NEAR_FAR = 0, FASTNERF_SAMPLES_IN_BOX = 1 } fastnerf_sample_mode;

typedef struct fastnerf_cache_s *fastnerf_cache;
typedef struct fastnerf_server_s *fastnerf_server;

typedef struct {
  int32_t k;                 /* voxels per axis, 1..4096 */
  int32_t D;                 /* components, 1..16 */
  int32_t l;                 /* direction cells per angle, 1..4096 */
  float bbox_min[3], bbox_max[3];
  fastnerf_dtype storage;    /* position-cache storage; beta is FP32 */
  fastnerf_interp pos_interp, dir_interp;
  int32_t brick;             /* occupancy brick edge in voxels (power of two, k % brick == 0,
                                k / brick <= 1024); 0 = no empty-space skipping */
  fastnerf_sample_mode sample_mode;
  float background[3];
  int32_t sparse;            /* 1: store only the 8^3 bricks that hold a voxel with sigma > 0
                                (the occupied bricks of the bitgrid); the others read as
                                zero. Needs nearest lookups, brick = 8 and k % 8 == 0.
                                0: every voxel is stored. [Sec. 1, supplementary "Meshing &
                                Rendering": the caches are stored sparsely] */
} fastnerf_cache_desc;

/* ---------------------------------------------------------------- caches */

/* Builds a cache from FP32 arrays (host or device): sigma[k][k][k] (index
 * (z*k + y)*k + x), u[k][k][k][D][3], beta[l][l][D] (theta row, phi column).
 * Quantises to desc->storage, builds the occupancy bitgrid (dilated by one
 * voxel for trilinear lookups) and returns a handle that is immutable and may
 * be rendered from several streams at once. Work is enqueued on `stream`; the
 * call returns after the input arrays have been consumed. [Sec. 3.3] */
fastnerf_status fastnerf_cache_create(const fastnerf_cache_desc *desc, const float *sigma,
                                      const float *u, const float *beta, hipStream_t stream,
                                      fastnerf_cache *out);

/* Slab-wise construction for caches larger than host memory or built on the
 * device: create_empty, then (FP8 or sparse caches) scan_slab for every slab
 * so that the per-channel scales and the stored bricks are known, then
 * upload_slab for every slab with the same data, then finalize, all on one
 * stream (or ordered by the caller). A slab is nz consecutive z layers
 * starting at z0, laid out like the full arrays. */
fastnerf_status fastnerf_cache_create_empty(const fastnerf_cache_desc *desc, const float *beta,
                                            hipStream_t stream, fastnerf_cache *out);
fastnerf_status fastnerf_cache_scan_slab(fastnerf_cache cache, int32_t z0, int32_t nz,
                                         const float *sigma, const float *u, hipStream_t stream);
fastnerf_status fastnerf_cache_upload_slab(fastnerf_cache cache, int32_t z0, int32_t nz,
                                           const float *sigma, const float *u, hipStream_t stream);
fastnerf_status fastnerf_cache_finalize(fastnerf_cache cache, hipStream_t stream);

/* Device bytes held by the cache (records, direction cache, bitgrid, distance
 * field, scales). */
fastnerf_status fastnerf_cache_bytes(fastnerf_cache cache, uint64_t *resident);
/* Bytes per stored voxel record (padded) and of its payload, (1+3D)*size(storage). */
fastnerf_status fastnerf_cache_record_bytes(fastnerf_cache cache, int32_t *stride,
                                            int32_t *payload);
/* Dequantised copy of the stored cache into caller device buffers
 * sigma[k^3] and u[k^3*D*3] (FP32), and the per-channel scales (host, 1+3D
 * floats, may be NULL). Synchronises `stream`. Test hook. */
fastnerf_status fastnerf_cache_readback(fastnerf_cache cache, float *sigma, float *u,
                                        float *scales, hipStream_t stream);
/* Occupancy bitgrid (host copy): nbricks^3 bits, brick index (bz*n + by)*n + bx,
 * bit b in word b/32. words must hold ceil(n^3/32) entries. */
fastnerf_status fastnerf_cache_occupancy(fastnerf_cache cache, uint32_t *words, int32_t *n);
/* Empty-space distance field (host copy, after finalize): one byte per
 * distance brick -- the bitgrid's brick, or 8^3 voxels when the bitgrid's is
 * smaller (and k a multiple of 8) -- in the bitgrid's brick order, holding the
 * max-norm (Chebyshev) distance in such bricks to the nearest one holding a
 * set bit: 0 for such a brick, capped at 63.
 * The renderer skips samples with it; output is unchanged by the skipping
 * (Sec. 4: the caches are sparse, empty space is never sampled). dist must hold
 * n^3 bytes; n receives the bricks per axis (0 without a bitgrid). Test hook. */
fastnerf_status fastnerf_cache_skip_distance(fastnerf_cache cache, uint8_t *dist, int32_t *n);
/* Waits for renders that use the cache, then frees it. */
fastnerf_status fastnerf_cache_destroy(fastnerf_cache cache);

/* ---------------------------------------------------------------- rendering */

/* Renders one H x W view into out (device, float[H][W][4]). N in [1, 4096]
 * samples per ray, or N = 0 to visit every voxel the ray crosses inside
 * [near, far] and the box, each with the length of the ray inside it (the
 * per-voxel integration of Sec. 4; nearest position lookups and k <= 1024,
 * EINVAL otherwise). near < far, eps in [0, 1). One persistent launch on
 * `stream`; asynchronous. [Sec. 3.1 Eq. 1, Sec. 3.2 Eq. 5, Sec. 4] */
fastnerf_status fastnerf_render(fastnerf_cache cache, const float K[9], const float c2w[12],
                                int32_t H, int32_t W, float near, float far, int32_t N, float eps,
                                float *out, hipStream_t stream);

/* Renders nviews views of one cache in a single persistent launch. K, c2w,
 * H, W, near, far and out are host arrays of nviews entries (out[i] is a
 * device buffer of H[i]*W[i]*4 floats). N as for fastnerf_render. The view
 * descriptors are staged through a ring of 8 pinned buffers per stream, so
 * the call returns without waiting for earlier launches; only a ninth batch
 * enqueued while the eighth-previous one's descriptor copy has not yet run on
 * the stream waits for that copy. Calls on one stream from several host
 * threads are serialised by the library. [Sec. 3.1 Eq. 1, Sec. 4] */
fastnerf_status fastnerf_render_batch(fastnerf_cache cache, int32_t nviews, const float *K,
                                      const float *c2w, const int32_t *H, const int32_t *W,
                                      const float *near, const float *far, int32_t N, float eps,
                                      float *const *out, hipStream_t stream);

/* fastnerf_render without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). Same arguments, checks, result and asynchrony as
 * fastnerf_render (images up to 65536 x 65536; N = 0 allowed); out is the
 * caller's device buffer. Its only scratch is the render's tile-queue
 * counters, 4 KiB in a fixed array in the library's device memory (one copy
 * per device, held until the process ends, its address looked up on the
 * device's first call), whatever the image size; each call clears them on
 * `stream` with a small kernel before the render. Every call on a device
 * shares that array: calls that overlap on one device (on different streams,
 * or from several host threads) race and must be ordered by the caller. */
fastnerf_status fastnerf_render_noalloc(fastnerf_cache cache, const float K[9],
                                        const float c2w[12], int32_t H, int32_t W, float near,
                                        float far, int32_t N, float eps, float *out,
                                        hipStream_t stream);

/* Scheduling of the fixed-N render launches (fastnerf_render,
 * fastnerf_render_batch, fastnerf_render_noalloc), process-wide. TILES: each
 * wave renders one 8x8 pixel tile at a time (one ray per lane) and takes the
 * next tile when all of its rays have stopped. REFILL: the wave-level ray
 * queue -- after each window of samples the wave takes a ballot of its live
 * lanes and, once enough have retired, refills them with set-up rays from a
 * per-wave pool in LDS, replenished a tile at a time (the rays of a tile that
 * miss the box are written at once, the others compacted into the pool).
 * WIDE: tiles with more records in flight per lane at fewer waves per SIMD,
 * which shortens the heaviest rays' dependency chains in launches too small
 * to fill the chip. SPLIT (single views of dense caches with nearest lookups
 * and D <= 8; other launches asked for it run WIDE): 4x4 pixel tiles with
 * four lanes per ray, which share each window's occupancy scan and gather
 * the window's occupied samples four at a time, one per lane; all four lanes
 * composite the samples in order. AUTO (the default): for launches of at
 * most 20,000 8x8 tiles (about two 800x800 views) SPLIT where it applies,
 * WIDE otherwise; TILES for larger launches. Every schedule gives bitwise the
 * same image: each sample's arithmetic and the order of the composite are the
 * same. Serving steps and voxel traversal (N = 0) use TILES. Returns EINVAL
 * for an unknown value. */
enum {
  FASTNERF_SCHEDULE_AUTO = 0,
  FASTNERF_SCHEDULE_TILES = 1,
  FASTNERF_SCHEDULE_REFILL = 2,
  FASTNERF_SCHEDULE_WIDE = 3,
  FASTNERF_SCHEDULE_SPLIT = 4
};
fastnerf_status fastnerf_set_schedule(int32_t schedule);
int32_t fastnerf_get_schedule(void);

/* Test hook: the kernel's own lookups. pts and dirs are device arrays of n
 * points / unit directions (3 floats each); sigma_u receives n*(1+3D) floats
 * (sigma then u[D][3]), beta n*D floats (device). */
fastnerf_status fastnerf_debug_lookup(fastnerf_cache cache, int32_t n, const float *pts,
                                      const float *dirs, float *sigma_u, float *beta,
                                      hipStream_t stream);

/* ---------------------------------------------------------------- memory model */

/* The paper's cache-size model (supplementary S4, Eq. S2):
 * alpha * (D*s_uvw + s_sigma) * k^3 + D * s_beta * l^2 bytes, where s_uvw is
 * the size of one stored (u_i, v_i, w_i) triple, s_sigma of a density and
 * s_beta of a weight, and alpha in [0, 1] is the occupied fraction. */
double fastnerf_model_bytes(double alpha, int64_t k, int64_t l, int32_t D, double s_sigma,
                            double s_uvw, double s_beta);

/* ---------------------------------------------------------------- serving */

/* A continuous-batching render server over resident caches. Requests are
 * admitted while their output fits the arena (bytes of device memory the
 * server owns; arena_bytes = 0 sizes it to a quarter of the device memory
 * free at creation, after the scenes are resident) and fewer than
 * max_inflight are running; every step renders
 * the running requests' tiles, an equal share each of a tile budget, in one
 * persistent launch per (storage format, lookup, component class) group,
 * replayed as a HIP graph on that group's own stream. Requests that arrive
 * while others run join at the next step. The server's streams, graphs and
 * pinned tables are created here and on a group's first use, and released by
 * destroy. */
fastnerf_status fastnerf_server_create(const fastnerf_cache *scenes, int32_t nscenes,
                                       uint64_t arena_bytes, int32_t max_inflight,
                                       fastnerf_server *out);
/* Non-blocking. N in [1, 4096] (no voxel traversal in serving steps).
 * EBUSY when the queue is full, ENOMEM when the request can never fit the
 * arena, ESHUTDOWN after destroy began. */
fastnerf_status fastnerf_serve_submit(fastnerf_server server, int32_t scene, const float K[9],
                                      const float c2w[12], int32_t H, int32_t W, float near,
                                      float far, int32_t N, float eps, uint64_t *ticket);
/* Waits up to timeout_us (-1: forever) for a ticket. On OK, *out_device points
 * at the H*W*4 floats of the result (valid until release) and *latency_ms is
 * submit-to-completion time. */
fastnerf_status fastnerf_serve_wait(fastnerf_server server, uint64_t ticket, int64_t timeout_us,
                                    const float **out_device, double *latency_ms);
fastnerf_status fastnerf_serve_release(fastnerf_server server, uint64_t ticket);
fastnerf_status fastnerf_serve_cancel(fastnerf_server server, uint64_t ticket);
/* Counters: steps run, requests completed, max requests in one step. */
fastnerf_status fastnerf_server_stats(fastnerf_server server, uint64_t *steps,
                                      uint64_t *completed, uint64_t *max_batch);
/* Drains running work, cancels queued requests, frees everything. */
fastnerf_status fastnerf_server_destroy(fastnerf_server server);

/* ---------------------------------------------------------------- cache bake */

/* Evaluates FastNeRF's two networks where the caches sample them (Sec. 3.2,
 * Eqs. 3-4; Sec. 3.3): the position network F_pos at the voxel centres of a
 * k^3 grid, the direction network F_dir at the (theta, phi) cell centres of an
 * l x l grid. Matrix products run on the matrix cores in binary16 with FP32
 * accumulation; the Fourier features are computed in FP64 and rounded to
 * binary16, every hidden activation is rounded to binary16, biases and the
 * output layer's activations are FP32.
 *
 * Network (Sec. 4 and its readings): features of a point x (3 coordinates):
 * feature 6j + a = sin(2^j pi x_a), feature 6j + 3 + a = cos(2^j pi x_a),
 * j < L; then `layers` fully connected ReLU layers of `hidden` units (layer
 * `skip` takes [previous activation, features], hidden units first), then a
 * linear output layer. Position outputs: sigma = max(o_0, 0), u[d][c] =
 * sigmoid(o_{1+3d+c}). Direction outputs: beta = softmax(o) over D. */
typedef struct fastnerf_mlp_s *fastnerf_mlp;

typedef struct {
  int32_t D;          /* components, 1..16 */
  int32_t pos_hidden; /* hidden width of F_pos: a multiple of 32 in [32, 384] */
  int32_t pos_layers; /* hidden layers of F_pos, 1..16 */
  int32_t pos_skip;   /* hidden layer in [1, pos_layers) that also takes the features; -1: none */
  int32_t pos_freqs;  /* Fourier frequencies L of the position features, 1..10 */
  int32_t dir_hidden; /* hidden width of F_dir: a multiple of 32 in [32, 384] */
  int32_t dir_layers; /* hidden layers of F_dir, 1..16 */
  int32_t dir_freqs;  /* Fourier frequencies of the direction features, 1..10 */
} fastnerf_mlp_desc;

/* Copies both networks' parameters to the current device. pos_params and
 * dir_params are host FP32 arrays holding, for every layer in order (hidden
 * layers, then the output layer), W[fan_in][fan_out] row-major then
 * b[fan_out]. Fan-ins: 6L for layer 0, hidden + 6L for the skip layer, hidden
 * otherwise; fan-outs: hidden, then 1 + 3D (F_pos) or D (F_dir). Weights are
 * rounded to binary16 (nearest even); biases stay FP32. EINVAL on a bad
 * descriptor or a non-finite parameter. */
fastnerf_status fastnerf_mlp_create(const fastnerf_mlp_desc *desc, const float *pos_params,
                                    const float *dir_params, fastnerf_mlp *out);
/* Number of FP32 values fastnerf_mlp_create reads from pos_params and
 * dir_params for this descriptor (-1 if the descriptor is invalid). */
int64_t fastnerf_mlp_param_count(const fastnerf_mlp_desc *desc, int32_t which /* 0 pos, 1 dir */);
/* F_pos at the centres of voxels z0..z0+nz-1 of a k^3 grid over the box
 * (voxel (x, y, z) at bbox_min + (i + 1/2) (bbox_max - bbox_min) / k per
 * axis). Writes device FP32 arrays laid out like a cache slab:
 * sigma[nz][k][k], u[nz][k][k][D][3] (x fastest), ready for
 * fastnerf_cache_upload_slab. Enqueued on `stream`. k in [1, 4096]. */
fastnerf_status fastnerf_bake_position(fastnerf_mlp mlp, int32_t k, const float bbox_min[3],
                                       const float bbox_max[3], int32_t z0, int32_t nz,
                                       float *sigma, float *u, hipStream_t stream);
/* F_dir at the centres of an l x l direction grid (theta = (j + 1/2) pi / l,
 * phi = (m + 1/2) 2 pi / l): device FP32 beta[l][l][D], the direction cache of
 * fastnerf_cache_create. l in [1, 4096]. */
fastnerf_status fastnerf_bake_direction(fastnerf_mlp mlp, int32_t l, float *beta,
                                        hipStream_t stream);
/* Waits for the network's outstanding bakes, then frees it. */
fastnerf_status fastnerf_mlp_destroy(fastnerf_mlp mlp);

/* ------------------------------------------------ direction filtering and LOD */

/* Smooths a direction-cache table beta[l][l][D] (theta row, phi column) with
 * a Gaussian of standard deviation `sigma` cells on each axis (Sec. 4 allows
 * smoothing the direction cache with a filter kernel, a Gaussian for one, to
 * soften view-dependent effects): out[j][m] = sum_{a,b} g(a) g(b) in[clamp(j+a)][(m+b)
 * mod l] with g(t) = exp(-t^2 / (2 sigma^2)) for |t| <= ceil(3 sigma),
 * normalised to sum 1 -- periodic in phi, the edge rows repeated in theta
 * (the lookup clamps theta the same way). Convex combinations stay convex, so
 * rows summing to 1 still do. sigma in [0, 10]; 0 copies. Device arrays;
 * beta_out must not overlap beta_in. Enqueued on `stream`. */
fastnerf_status fastnerf_filter_direction(const float *beta_in, int32_t l, int32_t D, float sigma,
                                          float *beta_out, hipStream_t stream);

/* Level-of-detail choice among caches of one scene at several resolutions
 * ks[0..n-1] over the same box (Sec. 5: smaller caches trade detail for speed
 * and memory like levels of detail): the coarsest level whose voxel edge
 * (longest box side / k) is at most `ratio` times the footprint of one pixel
 * at the box centre (distance from the camera to the centre / focal length
 * K[0]); the finest level if none is. Host only. Returns the index, or -1 for
 * bad arguments (n < 1, k < 1, ratio <= 0, K[0] <= 0, non-finite input). */
int32_t fastnerf_lod_select(const int32_t *ks, int32_t n, const float bbox_min[3],
                            const float bbox_max[3], const float K[9], const float c2w[12],
                            float ratio);

/* Thread-local message for the last non-OK status of this thread. */
const char *fastnerf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FASTNERF_H */
