// Direction-cache filtering and the level-of-detail choice among caches of
// several resolutions.
#include <hip/hip_runtime.h>
#include <math.h>

#include "fastnerf.h"
#include "fastnerf_internal.h"

using namespace fnr;

namespace {

constexpr int kMaxTaps = 31;  // radius ceil(3 sigma) <= 30

// One output element per thread: the separable Gaussian as a 2-D sum over
// the (2r+1)^2 taps, theta clamped, phi periodic. The weights are recomputed
// per thread from the same expression, so every thread uses the same values.
__global__ void k_filter_direction(const float *__restrict__ in, int l, int D, float sigma,
                                   int r, float *__restrict__ out) {
  const int64_t n = (int64_t)l * l * D;
  float g[2 * kMaxTaps + 1];
  float sum = 0.0f;
  for (int t = -r; t <= r; ++t) {
    const float v = expf(-(float)(t * t) / (2.0f * sigma * sigma));
    g[t + r] = v;
    sum += v;
  }
  const float inv = 1.0f / sum;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int d = (int)(e % D);
    const int64_t cell = e / D;
    const int j = (int)(cell / l), m = (int)(cell % l);
    float acc = 0.0f;
    for (int a = -r; a <= r; ++a) {
      const int jj = min(max(j + a, 0), l - 1);
      float row = 0.0f;
      for (int b = -r; b <= r; ++b) {
        int mm = (m + b) % l;
        if (mm < 0) mm += l;
        row = fmaf(g[b + r], in[((int64_t)jj * l + mm) * D + d], row);
      }
      acc = fmaf(g[a + r], row, acc);
    }
    out[e] = acc * inv * inv;
  }
}

}  // namespace

extern "C" fastnerf_status fastnerf_filter_direction(const float *beta_in, int32_t l, int32_t D,
                                                     float sigma, float *beta_out,
                                                     hipStream_t stream) {
  if (l < 1 || l > 4096) return fail(FASTNERF_EINVAL, "l = %d outside [1, 4096]", l);
  if (D < 1 || D > 16) return fail(FASTNERF_EINVAL, "D = %d outside [1, 16]", D);
  if (!(sigma >= 0.0f && sigma <= 10.0f)) return fail(FASTNERF_EINVAL, "sigma outside [0, 10]");
  if (!beta_in || !beta_out || !is_device_ptr(beta_in) || !is_device_ptr(beta_out))
    return fail(FASTNERF_EINVAL, "beta_in and beta_out must be device arrays");
  const uint64_t bytes = (uint64_t)l * l * D * sizeof(float);
  const uintptr_t a0 = (uintptr_t)beta_in, b0 = (uintptr_t)beta_out;
  if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(FASTNERF_EINVAL, "beta_out overlaps beta_in");
  if (sigma == 0.0f) {
    hipError_t e = hipMemcpyAsync(beta_out, beta_in, bytes, hipMemcpyDeviceToDevice, stream);
    return e == hipSuccess ? FASTNERF_OK : hip_fail(e, "copy");
  }
  const int r = (int)ceilf(3.0f * sigma);
  const int64_t n = (int64_t)l * l * D;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_filter_direction, dim3((unsigned)(blocks < 65536 ? blocks : 65536)),
                     dim3(256), 0, stream, beta_in, l, D, sigma, r, beta_out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FASTNERF_OK : hip_fail(e, "filter launch");
}

extern "C" int32_t fastnerf_lod_select(const int32_t *ks, int32_t n, const float bbox_min[3],
                                       const float bbox_max[3], const float K[9],
                                       const float c2w[12], float ratio) {
  if (!ks || n < 1 || !bbox_min || !bbox_max || !K || !c2w) return -1;
  if (!(ratio > 0.0f) || !isfinite(ratio) || !(K[0] > 0.0f) || !isfinite(K[0])) return -1;
  double side = 0.0, dist2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    if (!isfinite(bbox_min[a]) || !isfinite(bbox_max[a]) || !(bbox_min[a] < bbox_max[a]) ||
        !isfinite(c2w[4 * a + 3]))
      return -1;
    side = fmax(side, (double)bbox_max[a] - (double)bbox_min[a]);
    const double c = 0.5 * ((double)bbox_min[a] + (double)bbox_max[a]) - (double)c2w[4 * a + 3];
    dist2 += c * c;
  }
  const double footprint = sqrt(dist2) / (double)K[0];
  int best = -1, finest = -1;
  for (int i = 0; i < n; ++i) {
    if (ks[i] < 1) return -1;
    if (finest < 0 || ks[i] > ks[finest]) finest = i;
    if (side / ks[i] <= ratio * footprint && (best < 0 || ks[i] < ks[best])) best = i;
  }
  return best >= 0 ? best : finest;
}
