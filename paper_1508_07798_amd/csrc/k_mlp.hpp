// Rank-predictor MLP 8 -> 64 -> 64 -> 1 (tanh, tanh, linear), FP32.
// Parameter layout (HSS_MLP_NPARAMS floats): W1[64][8], b1[64], W2[64][64],
// b2[64], W3[1][64], b3[1] (row-major [out][in]).
// Loss: mean squared error of the prediction against log2(1 + rank).
#pragma once

#include "common.hpp"

namespace hss {

constexpr int MLP_IN = 8, MLP_H = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 512, OFF_W2 = 576, OFF_B2 = 4672, OFF_W3 = 4736, OFF_B3 = 4800;
constexpr int MLP_NP = 4801;

// one thread per sample: activations a1, a2 (n x 64 each, row-major) and y
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ w, const float* __restrict__ x,
                                                          int n, float* __restrict__ a1, float* __restrict__ a2,
                                                          float* __restrict__ y) {
  __shared__ float sw[MLP_NP];
  for (int i = threadIdx.x; i < MLP_NP; i += blockDim.x) sw[i] = w[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float in[MLP_IN], h1[MLP_H];
  for (int i = 0; i < MLP_IN; ++i) in[i] = x[s * MLP_IN + i];
  for (int o = 0; o < MLP_H; ++o) {
    float z = sw[OFF_B1 + o];
    for (int i = 0; i < MLP_IN; ++i) z += sw[OFF_W1 + o * MLP_IN + i] * in[i];
    h1[o] = tanhf(z);
    if (a1) a1[s * MLP_H + o] = h1[o];
  }
  float out = sw[OFF_B3];
  for (int o = 0; o < MLP_H; ++o) {
    float z = sw[OFF_B2 + o];
    for (int i = 0; i < MLP_H; ++i) z += sw[OFF_W2 + o * MLP_H + i] * h1[i];
    const float h2 = tanhf(z);
    if (a2) a2[s * MLP_H + o] = h2;
    out += sw[OFF_W3 + o] * h2;
  }
  y[s] = out;
}

// one thread per sample: dz2 = (2/n)(y - t) W3 * (1 - a2^2), dz1 = (dz2 W2) * (1 - a1^2),
// dy = (2/n)(y - t); the squared residuals go to r2
__global__ __launch_bounds__(256) void mlp_backward_kernel(const float* __restrict__ w, const float* __restrict__ y,
                                                           const float* __restrict__ t, int n,
                                                           const float* __restrict__ a1, const float* __restrict__ a2,
                                                           float* __restrict__ dz1, float* __restrict__ dz2,
                                                           float* __restrict__ dy, float* __restrict__ r2) {
  __shared__ float sw[MLP_NP];
  for (int i = threadIdx.x; i < MLP_NP; i += blockDim.x) sw[i] = w[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const float r = y[s] - t[s];
  r2[s] = r * r;
  const float g = 2.0f * r / (float)n;
  dy[s] = g;
  float d2[MLP_H];
  for (int o = 0; o < MLP_H; ++o) {
    const float h = a2[s * MLP_H + o];
    d2[o] = g * sw[OFF_W3 + o] * (1.0f - h * h);
    dz2[s * MLP_H + o] = d2[o];
  }
  for (int i = 0; i < MLP_H; ++i) {
    float acc = 0;
    for (int o = 0; o < MLP_H; ++o) acc += d2[o] * sw[OFF_W2 + o * MLP_H + i];
    const float h = a1[s * MLP_H + i];
    dz1[s * MLP_H + i] = acc * (1.0f - h * h);
  }
}

// one thread per parameter: sums over the samples (fixed order, deterministic)
__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* __restrict__ x, int n,
                                                       const float* __restrict__ a1, const float* __restrict__ a2,
                                                       const float* __restrict__ dz1, const float* __restrict__ dz2,
                                                       const float* __restrict__ dy, float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_NP) return;
  double acc = 0;
  if (p < OFF_B1) {
    const int o = p / MLP_IN, i = p % MLP_IN;
    for (int s = 0; s < n; ++s) acc += (double)dz1[s * MLP_H + o] * x[s * MLP_IN + i];
  } else if (p < OFF_W2) {
    const int o = p - OFF_B1;
    for (int s = 0; s < n; ++s) acc += dz1[s * MLP_H + o];
  } else if (p < OFF_B2) {
    const int o = (p - OFF_W2) / MLP_H, i = (p - OFF_W2) % MLP_H;
    for (int s = 0; s < n; ++s) acc += (double)dz2[s * MLP_H + o] * a1[s * MLP_H + i];
  } else if (p < OFF_W3) {
    const int o = p - OFF_B2;
    for (int s = 0; s < n; ++s) acc += dz2[s * MLP_H + o];
  } else if (p < OFF_B3) {
    const int i = p - OFF_W3;
    for (int s = 0; s < n; ++s) acc += (double)dy[s] * a2[s * MLP_H + i];
  } else {
    for (int s = 0; s < n; ++s) acc += dy[s];
  }
  grad[p] = (float)acc;
}

// sum of r2 / n into loss[0] (single workgroup)
__global__ __launch_bounds__(256) void mlp_loss_kernel(const float* __restrict__ r2, int n, float* __restrict__ loss) {
  __shared__ double red[256];
  double acc = 0;
  for (int s = threadIdx.x; s < n; s += 256) acc += r2[s];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(red[0] / n);
}

__global__ void mlp_adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, int t, float lr, float b1, float b2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_NP) return;
  const float gg = g[p];
  const float mm = b1 * m[p] + (1.0f - b1) * gg;
  const float vv = b2 * v[p] + (1.0f - b2) * gg * gg;
  m[p] = mm;
  v[p] = vv;
  const float mh = mm / (1.0f - powf(b1, (float)t));
  const float vh = vv / (1.0f - powf(b2, (float)t));
  w[p] -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace hss
