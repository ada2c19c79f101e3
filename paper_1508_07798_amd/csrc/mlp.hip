// Rank-predictor MLP entry points (forward, gradient, Adam training).
#include <hip/hip_runtime.h>

#include <vector>

#include "common.hpp"
#include "k_mlp.hpp"

namespace hss {

namespace {
struct MlpWork {
  float *a1, *a2, *dz1, *dz2, *dy, *r2, *y, *grad, *m, *v, *loss;
  std::vector<void*> owned;
  explicit MlpWork(int n, bool adam) {
    auto get = [&](size_t cnt) {
      void* p = nullptr;
      HIP_CHECK(hipMalloc(&p, std::max<size_t>(cnt, 1) * sizeof(float)));
      owned.push_back(p);
      return (float*)p;
    };
    a1 = get((size_t)n * MLP_H);
    a2 = get((size_t)n * MLP_H);
    dz1 = get((size_t)n * MLP_H);
    dz2 = get((size_t)n * MLP_H);
    dy = get(n);
    r2 = get(n);
    y = get(n);
    grad = get(MLP_NP);
    loss = get(1);
    m = adam ? get(MLP_NP) : nullptr;
    v = adam ? get(MLP_NP) : nullptr;
  }
  ~MlpWork() {
    for (void* p : owned) (void)hipFree(p);
  }
};

void check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(-5, std::string(what) + ": " + hipGetErrorString(e));
}

void grad_pass(const float* w, const float* x, const float* t, int n, MlpWork& wk, hipStream_t st) {
  const int blocks = (n + 255) / 256;
  mlp_forward_kernel<<<blocks, 256, 0, st>>>(w, x, n, wk.a1, wk.a2, wk.y);
  check("mlp_forward");
  mlp_backward_kernel<<<blocks, 256, 0, st>>>(w, wk.y, t, n, wk.a1, wk.a2, wk.dz1, wk.dz2, wk.dy, wk.r2);
  check("mlp_backward");
  mlp_grad_kernel<<<(MLP_NP + 255) / 256, 256, 0, st>>>(x, n, wk.a1, wk.a2, wk.dz1, wk.dz2, wk.dy, wk.grad);
  check("mlp_grad");
  mlp_loss_kernel<<<1, 256, 0, st>>>(wk.r2, n, wk.loss);
  check("mlp_loss");
}
}  // namespace

void mlp_forward(const float* w, const float* x, int n, float* y, hipStream_t st) {
  mlp_forward_kernel<<<(n + 255) / 256, 256, 0, st>>>(w, x, n, nullptr, nullptr, y);
  check("mlp_forward");
  HIP_CHECK(hipStreamSynchronize(st));
}

void mlp_grad(const float* w, const float* x, const float* t, int n, float* grad, double* loss, hipStream_t st) {
  MlpWork wk(n, false);
  grad_pass(w, x, t, n, wk, st);
  HIP_CHECK(hipMemcpyAsync(grad, wk.grad, sizeof(float) * MLP_NP, hipMemcpyDeviceToDevice, st));
  float l = 0;
  HIP_CHECK(hipMemcpyAsync(&l, wk.loss, sizeof(float), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  *loss = l;
}

void mlp_train(float* w, const float* x, const float* t, int n, int steps, float lr, float* loss_hist,
               hipStream_t st) {
  MlpWork wk(n, true);
  HIP_CHECK(hipMemsetAsync(wk.m, 0, sizeof(float) * MLP_NP, st));
  HIP_CHECK(hipMemsetAsync(wk.v, 0, sizeof(float) * MLP_NP, st));
  for (int s = 1; s <= steps; ++s) {
    grad_pass(w, x, t, n, wk, st);
    if (loss_hist) HIP_CHECK(hipMemcpyAsync(loss_hist + (s - 1), wk.loss, sizeof(float), hipMemcpyDeviceToDevice, st));
    mlp_adam_kernel<<<(MLP_NP + 255) / 256, 256, 0, st>>>(w, wk.grad, wk.m, wk.v, s, lr, 0.9f, 0.999f, 1e-8f);
    check("mlp_adam");
  }
  HIP_CHECK(hipStreamSynchronize(st));
}

}  // namespace hss
