// The learned tree / tile-size selector's network: a 3-layer perceptron
// F -> 64 -> 64 -> 1 with tanh hidden units, FP32, that predicts the log of
// a factorization's run time from the shape, tile size, tree and batch
// size.  Forward pass, gradient of the mean squared error over a batch of
// samples, and Adam steps, all on the GPU.
//
// Parameter vector (FP32, contiguous): W1 [H x F] row-major, b1 [H],
// W2 [H x H] row-major (W2[j][k]: hidden-1 unit k -> hidden-2 unit j), b2 [H],
// W3 [H], b3 [1].
//
// One wave per sample, lane j holding hidden unit j of both layers; the
// per-sample gradients are written out and summed over the samples by a
// second kernel (fixed order, FP64 accumulation), so results do not depend
// on scheduling.
#include <hip/hip_runtime.h>

#include "mlp.h"

namespace tqr {

namespace {

constexpr int H = kMlpHidden;
constexpr int F = kMlpFeatures;
constexpr int OW1 = 0, OB1 = OW1 + H * F, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H;
constexpr int P = OB3 + 1;
static_assert(P == kMlpParams, "parameter count");
constexpr int WPB = 4;  // samples (waves) per block

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// h1, h2 (per sample, H each) and y
__device__ __forceinline__ void forward_one(const float *__restrict__ w, const float *__restrict__ x, int lane,
                                            float *hs, float &h1, float &h2, float &y) {
  float z = w[OB1 + lane];
#pragma unroll
  for (int f = 0; f < F; f++) z = fmaf(w[OW1 + lane * F + f], x[f], z);
  h1 = tanhf(z);
  hs[lane] = h1;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  z = w[OB2 + lane];
  for (int k = 0; k < H; k++) z = fmaf(w[OW2 + lane * H + k], hs[k], z);
  h2 = tanhf(z);
  y = wave_sum_f(w[OW3 + lane] * h2) + w[OB3];
}

__global__ __launch_bounds__(64 * WPB) void fwd(const float *w, const float *X, int64_t B, float *Y) {
  __shared__ float hs[WPB][H];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t s = (int64_t)blockIdx.x * WPB + wv;
  if (s >= B) return;  // whole waves
  float h1, h2, y;
  forward_one(w, X + s * F, lane, hs[wv], h1, h2, y);
  if (lane == 0) Y[s] = y;
}

// Per-sample gradient of (y - t)^2 / B into G[s * P + ...], and the
// sample's squared error into E[s].
__global__ __launch_bounds__(64 * WPB) void grad_samples(const float *w, const float *X, const float *T, int64_t B,
                                                         float *G, float *E) {
  __shared__ float hs[WPB][H];
  __shared__ float ds[WPB][H];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t s = (int64_t)blockIdx.x * WPB + wv;
  if (s >= B) return;
  const float *x = X + s * F;
  float h1, h2, y;
  forward_one(w, x, lane, hs[wv], h1, h2, y);
  const float err = y - T[s];
  const float dy = 2.0f * err / (float)B;
  float *g = G + s * P;
  // output layer
  g[OW3 + lane] = dy * h2;
  if (lane == 0) {
    g[OB3] = dy;
    E[s] = err * err;
  }
  // hidden layer 2: dz2_j = dy W3_j (1 - h2_j^2)
  const float dz2 = dy * w[OW3 + lane] * (1.0f - h2 * h2);
  g[OB2 + lane] = dz2;
  for (int k = 0; k < H; k++) g[OW2 + lane * H + k] = dz2 * hs[wv][k];
  ds[wv][lane] = dz2;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // hidden layer 1: lane k, dz1_k = (sum_j W2[j][k] dz2_j) (1 - h1_k^2)
  float dh1 = 0.0f;
  for (int j = 0; j < H; j++) dh1 = fmaf(w[OW2 + j * H + lane], ds[wv][j], dh1);
  const float dz1 = dh1 * (1.0f - h1 * h1);
  g[OB1 + lane] = dz1;
#pragma unroll
  for (int f = 0; f < F; f++) g[OW1 + lane * F + f] = dz1 * x[f];
}

// grad[p] = sum over samples of G[s * P + p]; loss = sum of E
__global__ __launch_bounds__(256) void reduce_grad(const float *G, const float *E, int64_t B, float *grad,
                                                   float *loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < P) {
    double acc = 0.0;
    for (int64_t s = 0; s < B; s++) acc += (double)G[s * P + p];
    grad[p] = (float)acc;
  }
  if (p == P && loss) {
    double acc = 0.0;
    for (int64_t s = 0; s < B; s++) acc += (double)E[s];
    *loss = (float)(acc / (double)B);
  }
}

// Adam (Kingma and Ba, 2015), bias-corrected, step t >= 1.
__global__ __launch_bounds__(256) void adam(float *w, const float *g, float *m1, float *m2, int64_t t, float lr,
                                            float b1, float b2, float eps) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const float gi = g[p];
  const float a = b1 * m1[p] + (1.0f - b1) * gi;
  const float v = b2 * m2[p] + (1.0f - b2) * gi * gi;
  m1[p] = a;
  m2[p] = v;
  const float ah = a / (1.0f - powf(b1, (float)t));
  const float vh = v / (1.0f - powf(b2, (float)t));
  w[p] -= lr * ah / (sqrtf(vh) + eps);
}

__global__ void zero(float *x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0f;
}

}  // namespace

size_t mlp_work_bytes(int64_t B) {
  // per-sample gradients and squared errors; the summed gradient and Adam's
  // two moments (used by the fitting loop)
  return ((size_t)B * P + (size_t)B + 3 * (size_t)P) * sizeof(float);
}

hipError_t mlp_forward(const float *w, const float *X, int64_t B, float *Y, hipStream_t s) {
  hipLaunchKernelGGL(fwd, dim3((unsigned)((B + WPB - 1) / WPB)), dim3(64 * WPB), 0, s, w, X, B, Y);
  return hipGetLastError();
}

hipError_t mlp_grad(const float *w, const float *X, const float *T, int64_t B, float *grad, float *loss, void *work,
                    hipStream_t s) {
  float *G = static_cast<float *>(work);
  float *E = G + (size_t)B * P;
  hipLaunchKernelGGL(grad_samples, dim3((unsigned)((B + WPB - 1) / WPB)), dim3(64 * WPB), 0, s, w, X, T, B, G, E);
  hipLaunchKernelGGL(reduce_grad, dim3((P + 1 + 255) / 256), dim3(256), 0, s, G, E, B, grad, loss);
  return hipGetLastError();
}

hipError_t mlp_adam(float *w, const float *g, float *m1, float *m2, int64_t t, float lr, hipStream_t s) {
  hipLaunchKernelGGL(adam, dim3((P + 255) / 256), dim3(256), 0, s, w, g, m1, m2, t, lr, 0.9f, 0.999f, 1e-8f);
  return hipGetLastError();
}

hipError_t mlp_zero(float *x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(zero, dim3(64), dim3(256), 0, s, x, n);
  return hipGetLastError();
}

}  // namespace tqr
