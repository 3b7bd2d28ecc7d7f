// Measurement kernels for the roofline of the render's gathers (not part of
// the render library): the rate at which one GPU sustains reads of random
// 128-byte lines, the unit in which the render's record gathers reach HBM.
// Each wave draws a random region of region_bytes per round and its lanes
// read random lines inside it (the render's gathers are local in the same
// way: a tile's rays read nearby bricks), so the figure excludes the
// address-translation misses of lines spread over the whole buffer.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  // a 64-bit finaliser (multiply-xorshift) as the per-lane random source
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

// MODE 0: each lane reads its whole line (8 x 16 B), as an FP32 record is read;
// MODE 1: each lane reads 32 B of its line (one E4M3 record);
// MODE 2: the 8 lanes of a group read one line together (16 B each), for the
//         lines of the 8 lanes in turn.
template <int MODE>
__global__ void __launch_bounds__(256) k_line_gather(const float4 *__restrict__ buf,
                                                     uint64_t nregions, uint64_t lines_per_region,
                                                     int iters, uint64_t seed, float *sink) {
  const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t wave = tid >> 6;
  const int lane = (int)(threadIdx.x & 63u);
  float acc = 0.0f;
  for (int it = 0; it < iters; ++it) {
    const uint64_t region = mix64(seed ^ (wave * 0x9E3779B97F4A7C15ull + (uint64_t)it)) % nregions;
    const uint64_t h = mix64(seed * 31u ^ (tid * 0xD1B54A32D192ED03ull + (uint64_t)it));
    const uint64_t line = region * lines_per_region + h % lines_per_region;  // < nregions * lpr
    if (MODE == 0) {
      const float4 *p = buf + line * 8u;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float4 v = p[q];
        acc += v.x + v.y + v.z + v.w;
      }
    } else if (MODE == 1) {
      const float4 *p = buf + line * 8u + 2u * ((h >> 40) & 3u);
      const float4 a = p[0], b = p[1];
      acc += a.x + a.w + b.x + b.w;
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint64_t lq = __shfl(line, (lane & ~7) | q, 64);
        const float4 v = buf[lq * 8u + (uint64_t)(lane & 7)];
        acc += v.x + v.y + v.z + v.w;
      }
    }
  }
  if (acc == 1234.5f) sink[0] = acc;  // never true for a zeroed buffer; keeps the loads
}

}  // namespace

// Launches `blocks` blocks of 256 lanes, each lane reading `iters` random
// lines (mode 0/1/2 as above) of the first nregions * region_bytes bytes of
// buf (device memory of `bytes` bytes, 16-byte aligned, region_bytes a
// multiple of 128 and at most bytes). sink: one device float. Returns 0, or
// -1 on bad arguments, or the HIP error of the launch.
extern "C" int fnr_line_gather(const void *buf, uint64_t bytes, uint64_t region_bytes, int mode,
                               int blocks, int iters, uint64_t seed, float *sink,
                               hipStream_t stream) {
  if (!buf || !sink || bytes < 128 || region_bytes < 128 || region_bytes % 128 ||
      region_bytes > bytes || blocks < 1 || iters < 1 || mode < 0 || mode > 2)
    return -1;
  const uint64_t lpr = region_bytes / 128, nregions = (bytes / 128) / lpr;
  const float4 *b = static_cast<const float4 *>(buf);
  if (mode == 0)
    hipLaunchKernelGGL(k_line_gather<0>, dim3(blocks), dim3(256), 0, stream, b, nregions, lpr,
                       iters, seed, sink);
  else if (mode == 1)
    hipLaunchKernelGGL(k_line_gather<1>, dim3(blocks), dim3(256), 0, stream, b, nregions, lpr,
                       iters, seed, sink);
  else
    hipLaunchKernelGGL(k_line_gather<2>, dim3(blocks), dim3(256), 0, stream, b, nregions, lpr,
                       iters, seed, sink);
  return (int)hipGetLastError();
}
