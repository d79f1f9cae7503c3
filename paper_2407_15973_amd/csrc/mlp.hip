// Learned per-block precision selector: a 16-64-64-3 ReLU MLP on the 16 block
// features, trained with softmax cross-entropy and Adam, run in FP32 on the
// GPU. One wave evaluates one sample: lane j owns hidden unit j of both layers
// (row j of W1 and W2, column j of W2 for the backward pass); activations are
// broadcast with readlane. Per-wave gradient partials are summed in a fixed
// order by a second kernel, so training is run-to-run deterministic.
#include <math.h>

#include "device_util.hpp"
#include "internal.hpp"

namespace mpb {

constexpr int NIN = 16, NH = 64, NOUT = 3;
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NOUT * NH, NPARAM = OB3 + NOUT, OMU = NPARAM, OSIG = NPARAM + NIN;
static_assert(NPARAM == BJAC_MLP_NPARAM, "parameter count");

__device__ __forceinline__ float bcastf(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ float wsumf(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

struct Net {
  float w1[NIN], w2r[NH], b1, b2, w3[NOUT];
};

__device__ __forceinline__ void load_net(const float *blob, int j, Net &n) {
#pragma unroll
  for (int i = 0; i < NIN; ++i) n.w1[i] = blob[OW1 + j * NIN + i];
#pragma unroll
  for (int i = 0; i < NH; ++i) n.w2r[i] = blob[OW2 + j * NH + i];
  n.b1 = blob[OB1 + j];
  n.b2 = blob[OB2 + j];
#pragma unroll
  for (int c = 0; c < NOUT; ++c) n.w3[c] = blob[OW3 + c * NH + j];
}

// Forward of one sample in one wave. xn: normalised input (uniform).
__device__ __forceinline__ void forward1(const Net &n, const float (&xn)[NIN], const float *b3, float &z1, float &h1,
                                         float &z2, float &h2, float (&lg)[NOUT]) {
  z1 = n.b1;
#pragma unroll
  for (int i = 0; i < NIN; ++i) z1 = fmaf(n.w1[i], xn[i], z1);
  h1 = fmaxf(z1, 0.f);
  z2 = n.b2;
#pragma unroll
  for (int i = 0; i < NH; ++i) z2 = fmaf(n.w2r[i], bcastf(h1, i), z2);
  h2 = fmaxf(z2, 0.f);
#pragma unroll
  for (int c = 0; c < NOUT; ++c) lg[c] = wsumf(n.w3[c] * h2) + b3[c];
}

__device__ __forceinline__ void load_x(const float *blob, const float *feat, int64_t s, float (&xn)[NIN]) {
#pragma unroll
  for (int i = 0; i < NIN; ++i) xn[i] = (feat[s * NIN + i] - blob[OMU + i]) / blob[OSIG + i];
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *blob, const float *feat, int32_t n,
                                                          float *logits, uint8_t *tags) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6, nw = (gridDim.x * 256) >> 6;
  Net net;
  load_net(blob, lane, net);
  const float b3[NOUT] = {blob[OB3], blob[OB3 + 1], blob[OB3 + 2]};
  for (int s = wave; s < n; s += nw) {
    float xn[NIN], z1, h1, z2, h2, lg[NOUT];
    load_x(blob, feat, s, xn);
    forward1(net, xn, b3, z1, h1, z2, h2, lg);
    if (lane == 0) {
      if (logits)
        for (int c = 0; c < NOUT; ++c) logits[(int64_t)s * NOUT + c] = lg[c];
      if (tags) {
        // argmax; ties keep the higher precision (lower class index)
        const int best = (lg[1] > lg[0]) ? ((lg[2] > lg[1]) ? 2 : 1) : ((lg[2] > lg[0]) ? 2 : 0);
        tags[s] = (uint8_t)(best == 0 ? P64 : (best == 1 ? P32 : P16));
      }
    }
  }
}

// Per-wave partial gradient of the mean cross-entropy over this wave's samples.
__global__ __launch_bounds__(256) void mlp_backward_kernel(const float *blob, const float *feat,
                                                           const int32_t *labels, int32_t n, float *part,
                                                           float *loss_part) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6, nw = (gridDim.x * 256) >> 6;
  Net net;
  load_net(blob, lane, net);
  float w2c[NH];  // column `lane` of W2
#pragma unroll
  for (int j = 0; j < NH; ++j) w2c[j] = blob[OW2 + j * NH + lane];
  const float b3[NOUT] = {blob[OB3], blob[OB3 + 1], blob[OB3 + 2]};
  float gw1[NIN], gw2[NH], gb1 = 0.f, gb2 = 0.f, gw3[NOUT] = {0.f, 0.f, 0.f}, gb3[NOUT] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < NIN; ++i) gw1[i] = 0.f;
#pragma unroll
  for (int i = 0; i < NH; ++i) gw2[i] = 0.f;
  float lsum = 0.f;
  const float invn = 1.0f / (float)n;
  for (int s = wave; s < n; s += nw) {
    float xn[NIN], z1, h1, z2, h2, lg[NOUT];
    load_x(blob, feat, s, xn);
    forward1(net, xn, b3, z1, h1, z2, h2, lg);
    const int y = min(max(labels[s], 0), NOUT - 1);
    const float m = fmaxf(lg[0], fmaxf(lg[1], lg[2]));
    float e[NOUT], se = 0.f;
#pragma unroll
    for (int c = 0; c < NOUT; ++c) {
      e[c] = expf(lg[c] - m);
      se += e[c];
    }
    lsum += (m + logf(se)) - (y == 0 ? lg[0] : (y == 1 ? lg[1] : lg[2]));
    float g[NOUT];
#pragma unroll
    for (int c = 0; c < NOUT; ++c) g[c] = (e[c] / se - (c == y ? 1.f : 0.f)) * invn;
    // layer 3
#pragma unroll
    for (int c = 0; c < NOUT; ++c) {
      gw3[c] = fmaf(g[c], h2, gw3[c]);
      gb3[c] += g[c];
    }
    const float gh2 = (z2 > 0.f) ? (g[0] * net.w3[0] + g[1] * net.w3[1] + g[2] * net.w3[2]) : 0.f;
    // layer 2: dW2[lane][i] += gh2[lane] * h1[i]; gh1[lane] = sum_j gh2[j] W2[j][lane]
    float gh1 = 0.f;
#pragma unroll
    for (int i = 0; i < NH; ++i) {
      gw2[i] = fmaf(gh2, bcastf(h1, i), gw2[i]);
      gh1 = fmaf(bcastf(gh2, i), w2c[i], gh1);
    }
    gb2 += gh2;
    gh1 = (z1 > 0.f) ? gh1 : 0.f;
#pragma unroll
    for (int i = 0; i < NIN; ++i) gw1[i] = fmaf(gh1, xn[i], gw1[i]);
    gb1 += gh1;
  }
  float *P = part + (int64_t)wave * NPARAM;
#pragma unroll
  for (int i = 0; i < NIN; ++i) P[OW1 + lane * NIN + i] = gw1[i];
#pragma unroll
  for (int i = 0; i < NH; ++i) P[OW2 + lane * NH + i] = gw2[i];
  P[OB1 + lane] = gb1;
  P[OB2 + lane] = gb2;
#pragma unroll
  for (int c = 0; c < NOUT; ++c) P[OW3 + c * NH + lane] = gw3[c];
  if (lane < NOUT) P[OB3 + lane] = gb3[lane];
  if (lane == 0) loss_part[wave] = lsum * invn;
}

__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float *part, const float *loss_part, int32_t nwaves,
                                                         float *grad, float *loss) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < NPARAM) {
    float s = 0.f;
    for (int w = 0; w < nwaves; ++w) s += part[(int64_t)w * NPARAM + i];
    grad[i] = s;
  }
  if (i == 0 && loss) {
    float s = 0.f;
    for (int w = 0; w < nwaves; ++w) s += loss_part[w];
    *loss = s;
  }
}

__global__ __launch_bounds__(256) void adam_kernel(float *theta, const float *grad, float *m, float *v, float lr,
                                                   float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= NPARAM) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static int mlp_waves(int32_t n) {
  int w = (n + 3) / 4;
  if (w > 1024) w = 1024;
  return w < 1 ? 1 : w;
}

int launch_mlp_select(const float *feat, int32_t nb, const float *blob, uint8_t *tags, hipStream_t st) {
  if (!feat || !blob || !tags || nb < 1) return BJAC_EINVAL;
  const int waves = mlp_waves(nb);
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((waves + 3) / 4), dim3(256), 0, st, blob, feat, nb, nullptr, tags);
  MPB_HIP(hipGetLastError());
  return BJAC_OK;
}

}  // namespace mpb

using namespace mpb;

extern "C" int bjac_mlp_forward(const float *blob, const float *feat, int32_t n, float *logits, uint8_t *tags,
                                void *stream) {
  if (!blob || !feat || n < 1 || (!logits && !tags)) return BJAC_EINVAL;
  const int waves = mlp_waves(n);
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((waves + 3) / 4), dim3(256), 0, (hipStream_t)stream, blob, feat, n,
                     logits, tags);
  MPB_HIP(hipGetLastError());
  return BJAC_OK;
}

extern "C" int bjac_mlp_workspace_query(int32_t n, size_t *bytes) {
  if (n < 1 || !bytes) return BJAC_EINVAL;
  const int waves = ((mlp_waves(n) + 3) / 4) * 4;
  *bytes = (size_t)waves * NPARAM * sizeof(float) + 256 + (size_t)waves * sizeof(float);
  return BJAC_OK;
}

extern "C" int bjac_mlp_backward(const float *blob, const float *feat, const int32_t *labels, int32_t n,
                                 float *grad, float *loss, void *workspace, size_t workspace_bytes, void *stream) {
  if (!blob || !feat || !labels || n < 1 || !grad || !workspace) return BJAC_EINVAL;
  size_t need = 0;
  bjac_mlp_workspace_query(n, &need);
  if (workspace_bytes < need) return BJAC_ENOMEM;
  const int blocks = (mlp_waves(n) + 3) / 4, waves = blocks * 4;
  float *part = (float *)workspace;
  float *lpart = (float *)((uint8_t *)workspace + (((size_t)waves * NPARAM * sizeof(float) + 255) & ~size_t(255)));
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(mlp_backward_kernel, dim3(blocks), dim3(256), 0, st, blob, feat, labels, n, part, lpart);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, part, lpart, waves, grad,
                     loss);
  MPB_HIP(hipGetLastError());
  return BJAC_OK;
}

extern "C" int bjac_mlp_adam(float *blob, const float *grad, float *m, float *v, int32_t t, float lr, float b1,
                             float b2, float eps, void *stream) {
  if (!blob || !grad || !m || !v || t < 1) return BJAC_EINVAL;
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, blob, grad, m, v,
                     lr, b1, b2, eps, c1, c2);
  MPB_HIP(hipGetLastError());
  return BJAC_OK;
}
