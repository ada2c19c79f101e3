// Rank-predictor MLP entry points (forward, gradient, Adam training).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
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

// ---------------------------------------------------------------- weights files
// Binary layout: the 8 bytes "HSSMLP01", an int32 parameter count (HSS_MLP_NPARAMS),
// then the parameters as float32 (W1, b1, W2, b2, W3, b3, row-major [out][in]),
// all little-endian.
namespace {
const char kMagic[8] = {'H', 'S', 'S', 'M', 'L', 'P', '0', '1'};
}

void mlp_write(const char* path, const std::vector<float>& w) {
  FILE* f = std::fopen(path, "wb");
  if (!f) throw Error(HSS_EINVAL, std::string("cannot write ") + path);
  const int32_t cnt = (int32_t)w.size();
  const bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&cnt, 4, 1, f) == 1 &&
                  std::fwrite(w.data(), 4, w.size(), f) == w.size();
  if (std::fclose(f) != 0 || !ok) throw Error(HSS_EINVAL, std::string("write failed: ") + path);
}

std::vector<float> mlp_read(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) throw Error(HSS_EINVAL, std::string("cannot read ") + path);
  char mg[8];
  int32_t cnt = 0;
  std::vector<float> w(MLP_NP);
  bool ok = std::fread(mg, 1, 8, f) == 8 && std::memcmp(mg, kMagic, 8) == 0 && std::fread(&cnt, 4, 1, f) == 1 &&
            cnt == MLP_NP && std::fread(w.data(), 4, MLP_NP, f) == (size_t)MLP_NP;
  std::fclose(f);
  if (!ok) throw Error(HSS_EINVAL, std::string("not a rank-model weights file: ") + path);
  for (float v : w)
    if (!std::isfinite(v)) throw Error(HSS_EINVAL, std::string("non-finite weight in ") + path);
  return w;
}

// Train the rank predictor from host samples (features n x 8, ranks n) on the
// device and write its weights: weights drawn N(0, 1/fan_in) (biases 0) from a
// splitmix64 stream keyed by seed, targets log2(1 + rank), 1500 full-batch Adam
// steps at learning rate 3e-3 (the library's training kernels).
void rank_model_train(const float* feat, const float* rank, int n, const char* path, uint64_t seed) {
  std::vector<float> w(MLP_NP, 0.f), t(n);
  uint64_t st = seed;
  auto next = [&]() {
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  auto normal = [&]() {
    const double u1 = ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  };
  for (int i = 0; i < OFF_B1; ++i) w[i] = (float)(normal() / std::sqrt((double)MLP_IN));
  for (int i = OFF_W2; i < OFF_B2; ++i) w[i] = (float)(normal() / std::sqrt((double)MLP_H));
  for (int i = OFF_W3; i < OFF_B3; ++i) w[i] = (float)(normal() / std::sqrt((double)MLP_H));
  for (int i = 0; i < n; ++i) {
    if (!(rank[i] >= 0) || !std::isfinite(rank[i])) throw Error(HSS_EINVAL, "ranks must be finite and >= 0");
    t[i] = (float)std::log2(1.0 + (double)rank[i]);
  }
  for (int64_t i = 0; i < (int64_t)n * MLP_IN; ++i)
    if (!std::isfinite(feat[i])) throw Error(HSS_EINVAL, "features must be finite");
  float *dw = nullptr, *dx = nullptr, *dt = nullptr;
  HIP_CHECK(hipMalloc(&dw, sizeof(float) * MLP_NP));
  try {
    HIP_CHECK(hipMalloc(&dx, sizeof(float) * (size_t)n * MLP_IN));
    HIP_CHECK(hipMalloc(&dt, sizeof(float) * (size_t)n));
    HIP_CHECK(hipMemcpy(dw, w.data(), sizeof(float) * MLP_NP, hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(dx, feat, sizeof(float) * (size_t)n * MLP_IN, hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(dt, t.data(), sizeof(float) * (size_t)n, hipMemcpyHostToDevice));
    mlp_train(dw, dx, dt, n, 1500, 3e-3f, nullptr, nullptr);
    HIP_CHECK(hipMemcpy(w.data(), dw, sizeof(float) * MLP_NP, hipMemcpyDeviceToHost));
  } catch (...) {
    (void)hipFree(dw);
    if (dx) (void)hipFree(dx);
    if (dt) (void)hipFree(dt);
    throw;
  }
  (void)hipFree(dw);
  (void)hipFree(dx);
  (void)hipFree(dt);
  mlp_write(path, w);
}

}  // namespace hss
