// Cache bake: FastNeRF's position and direction networks (Sec. 3.2, Eqs. 3-4)
// evaluated at the points the caches sample (Sec. 3.3), on the matrix cores.
//
// A workgroup of four waves takes 128 points through every layer. The
// activations stay in LDS as binary16 (128 rows x 384 columns plus the Fourier
// features), the weights stream from L2 as ready-made MFMA fragments, and
// every layer is one 128 x n x k product by v_mfma_f32_32x32x16_f16 (binary16
// inputs, FP32 accumulation) computed transposed, out^T = W^T act^T, so that
// each lane's accumulators hold four consecutive output columns of one point
// and go back to LDS as one 8-byte store. Wave w owns the output column
// blocks w, w+4, w+8 of 32 columns for all 128 rows (four row blocks); the
// weight fragments of the next two k-steps are in flight while two are
// multiplied. After a layer the accumulators take the bias and the ReLU and
// go back to LDS as binary16; the output layer's raw values go to LDS as FP32
// and the heads (relu / sigmoid / softmax) are applied while they are
// written out.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <vector>

#include "fastnerf.h"
#include "fastnerf_internal.h"

namespace fnr {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kRows = 128;                  // points per workgroup
constexpr int kWaves = 4;
constexpr int kThreads = kWaves * 64;
constexpr int kMaxHidden = 384;
constexpr int kActStride = kMaxHidden + 8;  // halves per activation row (16-byte aligned rows)
constexpr int kFeat = 64;                   // feature columns: 6L <= 60, zero padded
constexpr int kFeatStride = kFeat + 8;
constexpr int kMaxBlk = 3;                  // 32-column output blocks per wave (384 / 32 / 4)
constexpr int kMaxLayers = 16;
constexpr int kRawStride = 68;              // floats per row of the output layer's raw values
constexpr int kMaxBias = kMaxLayers * kMaxHidden + 64;  // floats of bias per network

struct BakeLayer {
  const half8 *w;  // fragments [k-step][block][lane]: W rows 16s + 8(lane/32) + i, column lane%32
  int boff;        // offset of the bias (nblk * 32 floats, zero past the fan-out) in the net's biases
  int ks_h;        // k-steps (16 inputs each) over the previous activation
  int ks_f;        // then k-steps over the features (layer 0 and the skip layer)
  int nblk;        // 32-column output blocks
};

struct BakeArgs {
  BakeLayer L[kMaxLayers + 1];  // hidden layers, then the output layer
  const float *bias;            // every layer's bias, in order
  int nbias;
  int nlayers;
  int freqs;
  int D;
  int64_t npoints;
  int k, z0;                    // position grid: voxel centres of layers z0..
  double lo[3], h[3];
  int l;                        // direction grid
  float *out0, *out1;           // sigma, u | beta
};

// Sample point q: a voxel centre (x fastest) or a direction-cell centre
// (theta row, phi column), in FP64.
template <int MODE>
__device__ inline void point_of(const BakeArgs &a, int64_t q, double x[3]) {
  if (MODE == 0) {
    const int64_t kk = (int64_t)a.k * a.k;
    const int64_t iz = q / kk, rem = q - iz * kk;
    const int64_t iy = rem / a.k, ix = rem - iy * a.k;
    x[0] = a.lo[0] + ((double)ix + 0.5) * a.h[0];
    x[1] = a.lo[1] + ((double)iy + 0.5) * a.h[1];
    x[2] = a.lo[2] + ((double)(a.z0 + iz) + 0.5) * a.h[2];
  } else {
    const int64_t j = q / a.l, m = q - j * a.l;
    const double th = ((double)j + 0.5) * M_PI / a.l;
    const double ph = ((double)m + 0.5) * 2.0 * M_PI / a.l;
    x[0] = sin(th) * cos(ph);
    x[1] = sin(th) * sin(ph);
    x[2] = cos(th);
  }
}

// Activation fragments of k-steps s, s+1 for the four row blocks.
__device__ __forceinline__ void load_act(const BakeLayer &Ly, const _Float16 *act,
                                         const _Float16 *feat, int s, int mrow, int kq,
                                         half8 (&a0)[4], half8 (&a1)[4]) {
  const bool from_act = s < Ly.ks_h;
  const _Float16 *src = from_act ? act + 16 * s : feat + 16 * (s - Ly.ks_h);
  const int stride = from_act ? kActStride : kFeatStride;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const _Float16 *p = src + (32 * mb + mrow) * stride + kq;
    a0[mb] = *reinterpret_cast<const half8 *>(p);
    a1[mb] = *reinterpret_cast<const half8 *>(p + 16);
  }
}

// Weight fragments of k-steps s, s+1 of layer L for the wave's NB blocks.
template <int NB>
__device__ __forceinline__ void load_w(const BakeLayer &L, int wave, int lane, int s,
                                       half8 (&b0)[NB], half8 (&b1)[NB]) {
  const size_t stride = (size_t)L.nblk * 64;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const half8 *p = L.w + (size_t)s * stride + (size_t)(wave + kWaves * j) * 64 + lane;
    b0[j] = p[0];
    b1[j] = p[stride];
  }
}

template <int NB>
__device__ __forceinline__ void mfma_pair(const half8 (&b0)[NB], const half8 (&b1)[NB],
                                          const half8 (&a0)[4], const half8 (&a1)[4],
                                          f32x16 (&acc)[4][kMaxBlk]) {
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
      acc[mb][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(b0[j], a0[mb], acc[mb][j], 0, 0, 0);
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
      acc[mb][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(b1[j], a1[mb], acc[mb][j], 0, 0, 0);
}

// The weight pair a set reloads at virtual step v: this layer's step v, or
// past its end the next layer's step v - ks when the stream continues into
// it (chain), else this layer's last pair again (a valid address,
// never used).
template <int NB>
__device__ __forceinline__ void reload_w(const BakeLayer &Ly, const BakeLayer &next, bool chain,
                                         int wave, int lane, int v, half8 (&b0)[NB],
                                         half8 (&b1)[NB]) {
  const int ks = Ly.ks_h + Ly.ks_f;
  if (v < ks || !chain) {
    load_w<NB>(Ly, wave, lane, min(v, ks - 2), b0, b1);
  } else {
    const int nks = next.ks_h + next.ks_f;
    load_w<NB>(next, wave, lane, min(v - ks, nks - 2), b0, b1);
  }
}

// acc[mb][j] += (W block j of this wave)^T x (rows of block mb)^T over every
// k-step of the layer; NB blocks per wave, no per-block conditions. Two sets
// of weight and activation registers alternate (steps s, s+1 and s+2, s+3):
// a set is reloaded, two steps ahead, as soon as its products are issued, so
// a weight load has the other set's products to arrive. On entry the sets
// hold steps 0-3; with chain (next layer: same block count; ks a multiple of
// 4) they hold the next layer's steps 0-3 on return, so its weights arrive
// while this layer is written back. KSH/KSF > 0 fix the k-steps at compile
// time and unroll the loop completely: straight-line code lets the compiler
// wait for exactly the set in use (in a loop it waited for every load at the
// top of each iteration); KSH < 0 is the general loop.
template <int NB, int KSH, int KSF>
__device__ __forceinline__ void layer_gemm(const BakeLayer &Ly, const BakeLayer &next,
                                           bool chain, const _Float16 *act,
                                           const _Float16 *feat, int wave, int lane,
                                           half8 (&x0)[NB], half8 (&x1)[NB], half8 (&y0)[NB],
                                           half8 (&y1)[NB], f32x16 (&acc)[4][kMaxBlk]) {
  const int mrow = lane & 31, kq = (lane >> 5) * 8;
  constexpr bool kFixed = KSH >= 0;
  const int ks = kFixed ? KSH + KSF : Ly.ks_h + Ly.ks_f;  // even: widths are multiples of 32
  const int last = ks - 2;
  half8 ax0[4], ax1[4], ay0[4], ay1[4];
  load_act(Ly, act, feat, 0, mrow, kq, ax0, ax1);
  // both halves in every iteration, so that loads complete in one order on
  // every path (the wait before a set's products then spares the other set)
  int s = 0;
  auto body = [&](int s) {
    load_act(Ly, act, feat, min(s + 2, last), mrow, kq, ay0, ay1);
    __builtin_amdgcn_sched_barrier(0);  // activation reads go out first
    mfma_pair<NB>(x0, x1, ax0, ax1, acc);
    reload_w<NB>(Ly, next, chain, wave, lane, s + 4, x0, x1);
    // neither the compiler nor the scheduler moves anything across: the
    // reload stays between the two halves
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    load_act(Ly, act, feat, min(s + 4, last), mrow, kq, ax0, ax1);
    __builtin_amdgcn_sched_barrier(0);
    mfma_pair<NB>(y0, y1, ay0, ay1, acc);
    reload_w<NB>(Ly, next, chain, wave, lane, s + 6, y0, y1);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
  };
  if constexpr (kFixed) {
#pragma unroll
    for (int t = 0; t + 4 <= KSH + KSF; t += 4) body(t);
    s = (KSH + KSF) / 4 * 4;
  } else {
    for (; s + 4 <= ks; s += 4) body(s);
  }
  if (s < ks) mfma_pair<NB>(x0, x1, ax0, ax1, acc);  // ks = 4t + 2: the last pair
}

// layer_gemm with the k-steps of the common widths fixed at compile time.
template <int NB>
__device__ __forceinline__ void layer_gemm_any(const BakeLayer &Ly, const BakeLayer &next,
                                               bool chain, const _Float16 *act,
                                               const _Float16 *feat, int wave, int lane,
                                               half8 (&x0)[NB], half8 (&x1)[NB],
                                               half8 (&y0)[NB], half8 (&y1)[NB],
                                               f32x16 (&acc)[4][kMaxBlk]) {
#define FNR_GEMM(H, F)                                                                   \
  if (Ly.ks_h == (H) && Ly.ks_f == (F)) {                                                \
    layer_gemm<NB, H, F>(Ly, next, chain, act, feat, wave, lane, x0, x1, y0, y1, acc);   \
    return;                                                                              \
  }
  FNR_GEMM(0, 4)
  FNR_GEMM(24, 0)
  FNR_GEMM(24, 4)
  FNR_GEMM(16, 0)
  FNR_GEMM(16, 4)
  FNR_GEMM(8, 0)
  FNR_GEMM(8, 4)
#undef FNR_GEMM
  layer_gemm<NB, -1, -1>(Ly, next, chain, act, feat, wave, lane, x0, x1, y0, y1, acc);
}

template <int NB>
__device__ __forceinline__ void zero_acc(f32x16 (&acc)[4][kMaxBlk]) {
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mb][j][r] = 0.0f;
}

typedef _Float16 half4 __attribute__((ext_vector_type(4)));

// The hidden layers for a wave owning NB column blocks of each (NB = 0: the
// wave only joins the barriers). After a layer: bias + ReLU, binary16, into
// the activation rows. Accumulator element r of lane l (transposed product)
// is output column 8(r/4) + 4(l/32) + r%4 of the block, row l%32 of the row
// block.
template <int NB>
__device__ void hidden_layers(const BakeArgs &a, _Float16 *act, const _Float16 *feat,
                              const float *sbias, int wave, int lane) {
  const int mrow = lane & 31;
  half8 x0[NB > 0 ? NB : 1], x1[NB > 0 ? NB : 1], y0[NB > 0 ? NB : 1], y1[NB > 0 ? NB : 1];
  if constexpr (NB > 0) {
    const BakeLayer L0 = a.L[0];
    load_w<NB>(L0, wave, lane, 0, x0, x1);
    load_w<NB>(L0, wave, lane, min(2, L0.ks_h + L0.ks_f - 2), y0, y1);
  }
  for (int li = 0; li < a.nlayers; ++li) {
    const BakeLayer Ly = a.L[li];
    if constexpr (NB > 0) {
      f32x16 acc[4][kMaxBlk];
      zero_acc<NB>(acc);
      const bool more = li + 1 < a.nlayers;
      const BakeLayer Ln = a.L[more ? li + 1 : li];
      const bool chain = more && (Ly.ks_h + Ly.ks_f) % 4 == 0;
      layer_gemm_any<NB>(Ly, Ln, chain, act, feat, wave, lane, x0, x1, y0, y1, acc);
      if (more && !chain) {
        load_w<NB>(Ln, wave, lane, 0, x0, x1);
        load_w<NB>(Ln, wave, lane, min(2, Ln.ks_h + Ln.ks_f - 2), y0, y1);
      }
      __syncthreads();  // every wave has read this layer's input
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int nb = wave + kWaves * j;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int n = 32 * nb + 8 * g + 4 * (lane >> 5);
          const float4 bias = *reinterpret_cast<const float4 *>(sbias + Ly.boff + n);
#pragma unroll
          for (int mb = 0; mb < 4; ++mb) {
            half4 v;
            v[0] = (_Float16)fmaxf(acc[mb][j][4 * g + 0] + bias.x, 0.0f);
            v[1] = (_Float16)fmaxf(acc[mb][j][4 * g + 1] + bias.y, 0.0f);
            v[2] = (_Float16)fmaxf(acc[mb][j][4 * g + 2] + bias.z, 0.0f);
            v[3] = (_Float16)fmaxf(acc[mb][j][4 * g + 3] + bias.w, 0.0f);
            *reinterpret_cast<half4 *>(act + (32 * mb + mrow) * kActStride + n) = v;
          }
        }
      }
    } else {
      __syncthreads();
    }
    __syncthreads();
  }
}

template <int MODE>
__global__ void __launch_bounds__(kThreads) k_bake(BakeArgs a) {
  __shared__ __attribute__((aligned(16))) _Float16 act[kRows * kActStride];
  __shared__ __attribute__((aligned(16))) _Float16 feat[kRows * kFeatStride];
  __shared__ __attribute__((aligned(16))) float sbias[kMaxBias];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * kRows;

  if (tid < kRows) {
    // Fourier features of one row: sin and cos of pi x in FP64, then of
    // 2^j pi x by the double-angle identities sin 2t = 2 sin t cos t,
    // cos 2t = 1 - 2 sin^2 t (FP64: ten doublings keep the error near
    // 1e-13), rounded to binary16.
    int64_t q = row0 + tid;
    if (q >= a.npoints) q = a.npoints - 1;  // rows past the end repeat the last point
    double x[3], sn[3], cs[3];
    point_of<MODE>(a, q, x);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      sn[ax] = sinpi(x[ax]);
      cs[ax] = cospi(x[ax]);
    }
    _Float16 f[kFeat];
#pragma unroll
    for (int c = 0; c < kFeat; ++c) f[c] = (_Float16)0.0f;
#pragma unroll
    for (int j = 0; j < 10; ++j) {
      if (j < a.freqs) {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          f[6 * j + ax] = (_Float16)(float)sn[ax];
          f[6 * j + 3 + ax] = (_Float16)(float)cs[ax];
          const double s2 = 2.0 * sn[ax] * cs[ax];
          const double c2 = 1.0 - 2.0 * sn[ax] * sn[ax];
          sn[ax] = s2;
          cs[ax] = c2;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kFeat; c += 8) {
      half8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = f[c + e];
      *reinterpret_cast<half8 *>(feat + tid * kFeatStride + c) = v;
    }
  } else {
    for (int i = tid - kRows; i < a.nbias; i += kThreads - kRows) sbias[i] = a.bias[i];
  }
  __syncthreads();

  // hidden layers: the wave's blocks w, w+4, w+8 below nblk (wave-uniform)
  const int nblk_h = a.L[0].nblk;
  const int nmine = nblk_h > wave ? (nblk_h - wave + kWaves - 1) / kWaves : 0;
  if (nmine >= 3)
    hidden_layers<3>(a, act, feat, sbias, wave, lane);
  else if (nmine == 2)
    hidden_layers<2>(a, act, feat, sbias, wave, lane);
  else if (nmine == 1)
    hidden_layers<1>(a, act, feat, sbias, wave, lane);
  else
    hidden_layers<0>(a, act, feat, sbias, wave, lane);

  // output layer (at most two blocks: waves 0 and 1), raw FP32 values to LDS
  const BakeLayer Lo = a.L[a.nlayers];
  const int mrow = lane & 31;
  f32x16 acc[4][kMaxBlk];
  if (wave < Lo.nblk) {
    half8 x0[1], x1[1], y0[1], y1[1];
    load_w<1>(Lo, wave, lane, 0, x0, x1);
    load_w<1>(Lo, wave, lane, min(2, Lo.ks_h + Lo.ks_f - 2), y0, y1);
    zero_acc<1>(acc);
    layer_gemm_any<1>(Lo, Lo, false, act, feat, wave, lane, x0, x1, y0, y1, acc);
  }
  __syncthreads();  // the raw values overwrite the activations
  float *raw = reinterpret_cast<float *>(act);
  if (wave < Lo.nblk) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int n = 32 * wave + 8 * g + 4 * (lane >> 5);
      const float4 bias = *reinterpret_cast<const float4 *>(sbias + Lo.boff + n);
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        float4 v;
        v.x = acc[mb][0][4 * g + 0] + bias.x;
        v.y = acc[mb][0][4 * g + 1] + bias.y;
        v.z = acc[mb][0][4 * g + 2] + bias.z;
        v.w = acc[mb][0][4 * g + 3] + bias.w;
        *reinterpret_cast<float4 *>(raw + (32 * mb + mrow) * kRawStride + n) = v;
      }
    }
  }
  __syncthreads();
  const int D = a.D;
  if (MODE == 0) {
    const int nout = 1 + 3 * D;
    for (int e = tid; e < kRows * nout; e += kThreads) {
      const int r = e / nout, c = e - r * nout;
      const int64_t q = row0 + r;
      if (q >= a.npoints) continue;
      const float v = raw[r * kRawStride + c];
      if (c == 0)
        a.out0[q] = fmaxf(v, 0.0f);
      else
        a.out1[q * (3 * D) + (c - 1)] = 1.0f / (1.0f + expf(-v));
    }
  } else if (tid < kRows) {
    const int64_t q = row0 + tid;
    if (q < a.npoints) {
      const float *o = raw + tid * kRawStride;
      float mx = o[0];
      for (int d = 1; d < D; ++d) mx = fmaxf(mx, o[d]);
      float sum = 0.0f;
      for (int d = 0; d < D; ++d) sum += expf(o[d] - mx);
      const float inv = 1.0f / sum;
      for (int d = 0; d < D; ++d) a.out0[q * D + d] = expf(o[d] - mx) * inv;
    }
  }
}

bool valid_desc(const fastnerf_mlp_desc *d) {
  if (!d) return false;
  auto width_ok = [](int h) { return h >= 32 && h <= kMaxHidden && h % 32 == 0; };
  return d->D >= 1 && d->D <= 16 && width_ok(d->pos_hidden) && width_ok(d->dir_hidden) &&
         d->pos_layers >= 1 && d->pos_layers <= kMaxLayers && d->dir_layers >= 1 &&
         d->dir_layers <= kMaxLayers &&
         (d->pos_skip == -1 || (d->pos_skip >= 1 && d->pos_skip < d->pos_layers)) &&
         d->pos_freqs >= 1 && d->pos_freqs <= 10 && d->dir_freqs >= 1 && d->dir_freqs <= 10;
}

struct NetShape {
  int layers, hidden, skip, freqs, nout;
};

NetShape net_shape(const fastnerf_mlp_desc *d, int which) {
  return which == 0 ? NetShape{d->pos_layers, d->pos_hidden, d->pos_skip, d->pos_freqs, 1 + 3 * d->D}
                    : NetShape{d->dir_layers, d->dir_hidden, -1, d->dir_freqs, d->D};
}

// Fan-in of the previous activation and whether the layer takes the features.
void layer_inputs(const NetShape &n, int i, int *hh, bool *feats, int *fan_out) {
  *hh = i == 0 ? 0 : n.hidden;
  *feats = i == 0 || i == n.skip;
  *fan_out = i == n.layers ? n.nout : n.hidden;
}

int64_t param_count(const NetShape &n) {
  int64_t c = 0;
  for (int i = 0; i <= n.layers; ++i) {
    int hh, fo;
    bool f;
    layer_inputs(n, i, &hh, &f, &fo);
    c += (int64_t)(hh + (f ? 6 * n.freqs : 0)) * fo + fo;
  }
  return c;
}

}  // namespace
}  // namespace fnr

using namespace fnr;

struct fastnerf_mlp_s {
  fastnerf_mlp_desc desc;
  int device = 0;
  uint8_t *buf = nullptr;
  fnr::BakeLayer net[2][fnr::kMaxLayers + 1];
  const float *bias[2] = {nullptr, nullptr};  // each network's biases (device)
  int nbias[2] = {0, 0};
  hipEvent_t last_use = nullptr;
};

extern "C" int64_t fastnerf_mlp_param_count(const fastnerf_mlp_desc *desc, int32_t which) {
  if (!valid_desc(desc) || (which != 0 && which != 1)) return -1;
  return param_count(net_shape(desc, which));
}

extern "C" fastnerf_status fastnerf_mlp_create(const fastnerf_mlp_desc *desc,
                                               const float *pos_params, const float *dir_params,
                                               fastnerf_mlp *out) {
  if (!out) return fail(FASTNERF_EINVAL, "null out");
  *out = nullptr;
  if (!valid_desc(desc)) return fail(FASTNERF_EINVAL, "invalid network descriptor");
  if (!pos_params || !dir_params) return fail(FASTNERF_EINVAL, "null parameters");
  if (is_device_ptr(pos_params) || is_device_ptr(dir_params))
    return fail(FASTNERF_EINVAL, "network parameters must be host arrays");
  const float *params[2] = {pos_params, dir_params};
  // pack every layer's weight fragments (binary16, 256-byte aligned), then
  // each network's biases (every layer padded to nblk * 32 floats), all in
  // one device buffer
  std::vector<uint8_t> host;
  std::vector<size_t> woff[2];
  std::vector<float> biases[2];
  int shape_ks[2][kMaxLayers + 1][4];
  for (int which = 0; which < 2; ++which) {
    const NetShape n = net_shape(desc, which);
    const int64_t count = param_count(n);
    for (int64_t i = 0; i < count; ++i)
      if (!isfinite(params[which][i])) return fail(FASTNERF_EINVAL, "non-finite parameter");
    const float *p = params[which];
    for (int i = 0; i <= n.layers; ++i) {
      int hh, fo;
      bool f;
      layer_inputs(n, i, &hh, &f, &fo);
      const int fan_in = hh + (f ? 6 * n.freqs : 0);
      const float *W = p, *b = p + (size_t)fan_in * fo;
      p = b + fo;
      const int ks_h = hh / 16, ks_f = f ? kFeat / 16 : 0, ks = ks_h + ks_f;
      const int nblk = (fo + 31) / 32;
      shape_ks[which][i][0] = ks_h;
      shape_ks[which][i][1] = ks_f;
      shape_ks[which][i][2] = nblk;
      shape_ks[which][i][3] = (int)biases[which].size();
      const size_t w0 = (host.size() + 255) & ~(size_t)255;
      host.resize(w0 + (size_t)ks * nblk * 64 * 16, 0);
      _Float16 *wf = reinterpret_cast<_Float16 *>(host.data() + w0);
      for (int s = 0; s < ks; ++s)
        for (int nb = 0; nb < nblk; ++nb)
          for (int l = 0; l < 64; ++l)
            for (int e = 0; e < 8; ++e) {
              const int kk = 16 * s + 8 * (l / 32) + e;  // input index of the padded layer
              int row = -1;
              if (s < ks_h) {
                row = kk;
              } else {
                const int fi = kk - 16 * ks_h;  // feature index
                if (fi < 6 * n.freqs) row = hh + fi;
              }
              const int col = 32 * nb + (l & 31);
              const float v = (row >= 0 && col < fo) ? W[(size_t)row * fo + col] : 0.0f;
              wf[(((size_t)s * nblk + nb) * 64 + l) * 8 + e] = (_Float16)v;
            }
      woff[which].push_back(w0);
      const size_t b0 = biases[which].size();
      biases[which].resize(b0 + (size_t)nblk * 32, 0.0f);
      memcpy(biases[which].data() + b0, b, (size_t)fo * 4);
    }
  }
  size_t boff[2];
  for (int which = 0; which < 2; ++which)
    if (biases[which].size() > (size_t)kMaxBias) return fail(FASTNERF_EINVAL, "too many biases");
  for (int which = 0; which < 2; ++which) {
    boff[which] = (host.size() + 255) & ~(size_t)255;
    host.resize(boff[which] + biases[which].size() * 4, 0);
    memcpy(host.data() + boff[which], biases[which].data(), biases[which].size() * 4);
  }
  fastnerf_mlp_s *m = new (std::nothrow) fastnerf_mlp_s();
  if (!m) return fail(FASTNERF_ENOMEM, "host allocation");
  m->desc = *desc;
  (void)hipGetDevice(&m->device);
  hipError_t e = hipMalloc(&m->buf, host.size());
  if (e == hipSuccess) e = hipMemcpy(m->buf, host.data(), host.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&m->last_use, hipEventDisableTiming);
  if (e != hipSuccess) {
    fastnerf_status st = hip_fail(e, "network upload");
    fastnerf_mlp_destroy(m);
    return st;
  }
  for (int which = 0; which < 2; ++which) {
    m->bias[which] = reinterpret_cast<const float *>(m->buf + boff[which]);
    m->nbias[which] = (int)biases[which].size();
    for (size_t i = 0; i < woff[which].size(); ++i) {
      BakeLayer &L = m->net[which][i];
      L.w = reinterpret_cast<const half8 *>(m->buf + woff[which][i]);
      L.ks_h = shape_ks[which][i][0];
      L.ks_f = shape_ks[which][i][1];
      L.nblk = shape_ks[which][i][2];
      L.boff = shape_ks[which][i][3];
    }
  }
  *out = m;
  return FASTNERF_OK;
}

static fastnerf_status launch_bake(fastnerf_mlp m, int which, BakeArgs &a, hipStream_t s) {
  const fastnerf_mlp_desc &d = m->desc;
  const NetShape n = net_shape(&d, which);
  for (int i = 0; i <= n.layers; ++i) a.L[i] = m->net[which][i];
  a.bias = m->bias[which];
  a.nbias = m->nbias[which];
  a.nlayers = n.layers;
  a.freqs = n.freqs;
  a.D = d.D;
  const int64_t blocks = (a.npoints + kRows - 1) / kRows;
  if (blocks > 0x7fffffffLL) return fail(FASTNERF_EINVAL, "too many points in one bake");
  if (which == 0)
    hipLaunchKernelGGL(k_bake<0>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_bake<1>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "bake launch");
  e = hipEventRecord(m->last_use, s);
  if (e != hipSuccess) return hip_fail(e, "bake event");
  return FASTNERF_OK;
}

extern "C" fastnerf_status fastnerf_bake_position(fastnerf_mlp m, int32_t k,
                                                  const float bbox_min[3],
                                                  const float bbox_max[3], int32_t z0, int32_t nz,
                                                  float *sigma, float *u, hipStream_t stream) {
  if (!m) return fail(FASTNERF_EINVAL, "null network");
  if (k < 1 || k > 4096) return fail(FASTNERF_EINVAL, "k = %d outside [1, 4096]", k);
  if (!bbox_min || !bbox_max) return fail(FASTNERF_EINVAL, "null bounding box");
  for (int ax = 0; ax < 3; ++ax)
    if (!isfinite(bbox_min[ax]) || !isfinite(bbox_max[ax]) || !(bbox_min[ax] < bbox_max[ax]))
      return fail(FASTNERF_EINVAL, "bad bounding box");
  if (z0 < 0 || nz < 1 || z0 + nz > k)
    return fail(FASTNERF_EINVAL, "slab [%d, %d) outside [0, %d)", z0, z0 + nz, k);
  if (!sigma || !u || !is_device_ptr(sigma) || !is_device_ptr(u))
    return fail(FASTNERF_EINVAL, "sigma and u must be device arrays");
  BakeArgs a;
  memset(&a, 0, sizeof a);
  a.npoints = (int64_t)nz * k * k;
  a.k = k;
  a.z0 = z0;
  for (int ax = 0; ax < 3; ++ax) {
    a.lo[ax] = bbox_min[ax];
    a.h[ax] = ((double)bbox_max[ax] - (double)bbox_min[ax]) / k;
  }
  a.out0 = sigma;
  a.out1 = u;
  return launch_bake(m, 0, a, stream);
}

extern "C" fastnerf_status fastnerf_bake_direction(fastnerf_mlp m, int32_t l, float *beta,
                                                   hipStream_t stream) {
  if (!m) return fail(FASTNERF_EINVAL, "null network");
  if (l < 1 || l > 4096) return fail(FASTNERF_EINVAL, "l = %d outside [1, 4096]", l);
  if (!beta || !is_device_ptr(beta)) return fail(FASTNERF_EINVAL, "beta must be a device array");
  BakeArgs a;
  memset(&a, 0, sizeof a);
  a.npoints = (int64_t)l * l;
  a.l = l;
  a.out0 = beta;
  return launch_bake(m, 1, a, stream);
}

extern "C" fastnerf_status fastnerf_mlp_destroy(fastnerf_mlp m) {
  if (!m) return fail(FASTNERF_EINVAL, "null network");
  if (m->last_use) {
    (void)hipEventSynchronize(m->last_use);
    (void)hipEventDestroy(m->last_use);
  }
  if (m->buf) (void)hipFree(m->buf);
  delete m;
  return FASTNERF_OK;
}
