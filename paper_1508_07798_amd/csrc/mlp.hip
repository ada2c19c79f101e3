// Rank-predictor MLP entry points (forward, gradient, Adam training).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hss.h"

#include "common.hpp"
#include "k_mlp.hpp"

namespace hss {

namespace {
// Device buffers of one gradient pass (activations, back-propagated terms, the
// prediction, the gradient, the loss) and, for training, Adam's moments.
struct MlpBufs {
  float *a1 = nullptr, *a2 = nullptr, *dz1 = nullptr, *dz2 = nullptr, *dy = nullptr, *r2 = nullptr,
        *y = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr;
  // carve the buffers for n samples out of consecutive floats starting at base
  // (returns the floats used); grad may point elsewhere
  size_t carve(float* base, int n, bool adam) {
    size_t off = 0;
    auto get = [&](size_t cnt) {
      float* p = base + off;
      off += (std::max<size_t>(cnt, 1) + 63) & ~size_t(63);  // 256-byte aligned pieces
      return p;
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
    return off;
  }
};
// the buffers in one device allocation of the library
struct MlpWork : MlpBufs {
  void* mem = nullptr;
  MlpWork(int n, bool adam) {
    const size_t floats = carve(nullptr, n, adam);
    HIP_CHECK(hipMalloc(&mem, floats * sizeof(float)));
    carve((float*)mem, n, adam);
  }
  ~MlpWork() {
    if (mem) (void)hipFree(mem);
  }
};

// The allocation-free gradient keeps its buffers in a fixed device array: the
// gradient pass for up to kMlpNoAllocMaxN samples. The array's device address is
// looked up once per device (hipGetSymbolAddress, with that device current) and
// kept; host code uses only that address, never the array's name.
constexpr int kMlpNoAllocMaxN = 8192;
constexpr size_t kMlpScratchFloats = 4 * ((size_t)kMlpNoAllocMaxN * MLP_H + 64) + 3 * ((size_t)kMlpNoAllocMaxN + 64) +
                                     (MLP_NP + 64) + 64;
__device__ __align__(256) float scratch[kMlpScratchFloats];
std::mutex g_scratch_mu;
std::vector<float*> g_scratch_ptr;  // per device ordinal

float* scratch_address() {
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error(HSS_EDEVICE, std::string("device address of the MLP scratch array: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (float*)p;
  }
  return g_scratch_ptr[dev];
}

void check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(-5, std::string(what) + ": " + hipGetErrorString(e));
}

void grad_pass(const float* w, const float* x, const float* t, int n, const MlpBufs& wk, hipStream_t st) {
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

int mlp_noalloc_max_n() { return kMlpNoAllocMaxN; }

// The gradient of mlp_grad with every buffer in the fixed device array: no device
// allocation. Calls on one device share the array, so calls that overlap on one
// device race; the kernels overwrite every buffer they read, nothing needs clearing.
void mlp_grad_noalloc(const float* w, const float* x, const float* t, int n, float* grad, double* loss,
                      hipStream_t st) {
  if (n > kMlpNoAllocMaxN)
    throw Error(HSS_EINVAL, "hss_mlp_grad_noalloc takes at most " + std::to_string(kMlpNoAllocMaxN) + " samples");
  MlpBufs wk;
  const size_t used = wk.carve(scratch_address(), n, false);
  if (used > kMlpScratchFloats) throw Error(HSS_EINVAL, "MLP scratch array too small");
  wk.grad = grad;  // the caller's output
  grad_pass(w, x, t, n, wk, st);
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
