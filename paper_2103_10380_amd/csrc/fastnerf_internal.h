// Host-side state shared by the library's translation units.
#pragma once
#include <stdint.h>

#include "fastnerf.h"
#include "fastnerf_device.h"

struct fastnerf_cache_s {
  fastnerf_cache_desc desc;
  int device = 0;
  uint8_t *rec = nullptr;      // records, brick-linear, stride bytes each (brick-sparse: the
                               // all-zero brick, then the stored bricks in brick order)
  float *beta = nullptr;       // [l][l][D]
  uint32_t *occ = nullptr;     // occupancy bits
  uint8_t *dist = nullptr;     // per-brick Chebyshev distance to the nearest occupied brick
  // brick-sparse caches: flags set by scan_slab, then the stored-brick slots
  // (0 = the all-zero brick) and, per bitgrid word, the set bits before it
  uint32_t *bflag = nullptr;
  int32_t *slot = nullptr;
  uint32_t *rank = nullptr;
  uint64_t nstored = 0;
  bool scanned = false, sparse_ready = false;
  float *scales = nullptr;     // 1 + 3D
  unsigned *amax = nullptr;    // FP8 absmax accumulators (float bits)
  int stride = 0, payload = 0, rec_shift = 0, nchunk = 0;
  int nbl = 0, nbo = 0, oshift = 0;
  int nbd = 0, dshift = 0;      // distance-field bricks per axis, log2 edge (>= the bitgrid's)
  uint64_t resident = 0, occ_bytes = 0;
  bool scales_ready = false, finalized = false;
  hipEvent_t last_use = nullptr;
};

namespace fnr {

fastnerf_status fail(fastnerf_status st, const char *fmt, ...);
fastnerf_status hip_fail(hipError_t e, const char *what);
bool is_device_ptr(const void *p);

struct StreamState;
fastnerf_status stream_state(hipStream_t s, StreamState **out);
DevCache dev_cache(const fastnerf_cache_s *c);
void make_view(const fastnerf_cache_s *c, const float K[9], const float c2w[12], int H, int W,
               float near_, float far_, float *out, int tile_begin, DevView *v);
fastnerf_status check_render_params(int N, float eps);
fastnerf_status check_view(const float *K, const float *c2w, int H, int W, float near_,
                           float far_, const float *out);
float eps_limit(float eps);

}  // namespace fnr
