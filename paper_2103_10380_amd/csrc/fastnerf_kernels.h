// Launchers of the gfx950 kernels (internal to the library).
#pragma once
#include "fastnerf_device.h"

namespace fnr {

// Resident blocks per CU of the render kernel (0 if it cannot launch):
// brick-sparse or dense cache, schedule kSched*.
int render_occupancy(int fmt, bool lin, int D, bool sparse, int sched, int occ_words);
// Threads per block of that kernel: kBlock, or one CU's worth for the tile
// kernel that stages the bitgrid (occ_words 32-bit words) in LDS.
int render_block(int fmt, bool lin, int D, bool sparse, int sched, int occ_words);
// Tile queues of a render launch and the spacing of their counters (uints):
// the counter buffer of a stream holds kQueueCounters uints.
constexpr int kQueueCounters = 32 * 32;
int render_step_occupancy(int fmt, bool lin, int D);
hipError_t launch_render_step(int fmt, bool lin, int D, const RenderArgs &a, int grid,
                              hipStream_t s);
hipError_t launch_render(int fmt, bool lin, const RenderArgs &a, int grid, hipStream_t s);
// Voxel traversal (views with N = 0; nearest lookups, k <= 1024).
int render_vox_occupancy(int fmt, int D);
hipError_t launch_render_vox(int fmt, const RenderArgs &a, int grid, hipStream_t s);
hipError_t launch_absmax(const float *sigma, const float *u, int64_t nvox, int D, unsigned *amax,
                         hipStream_t s);
hipError_t launch_fill_u32(unsigned *p, int n, unsigned v, hipStream_t s);
hipError_t launch_make_scales(const unsigned *amax, int nch, float *scales, hipStream_t s);
hipError_t launch_pack(int fmt, const float *sigma, const float *u, int z0, int nz,
                       const DevCache &c, hipStream_t s);
hipError_t launch_occupancy(int fmt, const DevCache &c, int dilate, uint32_t *words,
                            hipStream_t s);
// Brick-sparse caches: flags of the 8^3 bricks holding a voxel with sigma != 0.
hipError_t launch_brick_flags(const float *sigma, int z0, int nz, int k, int nbl,
                              uint32_t *flags, hipStream_t s);
// Per-brick distance field from the occupancy bits: dist[b] = Chebyshev
// distance in bricks to the nearest occupied brick, capped at kDistCap. tmp
// holds nbo^3 bytes of scratch.
hipError_t launch_distance(const DevCache &c, const uint32_t *words, uint8_t *dist, uint8_t *tmp,
                           hipStream_t s);
hipError_t launch_readback(int fmt, const DevCache &c, float *sigma, float *u, hipStream_t s);
hipError_t launch_lookup(int fmt, bool lin, const DevCache &c, int n, const float *pts,
                         const float *dirs, float *su, float *bo, hipStream_t s);

}  // namespace fnr
