// Host-only stand-ins for the device parts of libhss, so that the C ABI and the
// planner can be built with the host sanitizers (AddressSanitizer,
// UndefinedBehaviorSanitizer) and driven through hss_plan_* without a GPU. Every
// device entry reports HSS_EDEVICE.
#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "../../include/hss.h"
#include "../../paper_1508_07798_amd/csrc/common.hpp"
#include "../../paper_1508_07798_amd/csrc/engine.hpp"

namespace hss {
[[noreturn]] static void no_device() { throw Error(HSS_EDEVICE, "device code is not part of the sanitizer build"); }
std::unique_ptr<EngineBase> make_engine(std::shared_ptr<const Plan>, const hss_opts_t&, bool) { no_device(); }
void mlp_forward(const float*, const float*, int, float*, hipStream_t) { no_device(); }
void mlp_grad(const float*, const float*, const float*, int, float*, double*, hipStream_t) { no_device(); }
void mlp_train(float*, const float*, const float*, int, int, float, float*, hipStream_t) { no_device(); }
void mlp_grad_noalloc(const float*, const float*, const float*, int, float*, double*, hipStream_t) { no_device(); }
int mlp_noalloc_max_n() { return 8192; }
int panel_candidates(int, int, int32_t*, int) { return 0; }
std::vector<float> mlp_read(const char*) { no_device(); }
void rank_model_train(const float*, const float*, int, const char*, uint64_t) { no_device(); }
void debug_gemm(int, int, const void* const*, const void* const*, void* const*, const int32_t*, const int32_t*,
                const int32_t*, const int32_t*, const int32_t*, const int32_t*, const double*, const double*,
                hipStream_t) {
  no_device();
}
void debug_gj(int, int, void* const*, const int32_t*, const int32_t*, int, int32_t*, hipStream_t) { no_device(); }
void debug_row_id(int, const void*, int, int, double, int, int32_t*, int32_t*, void*, float*, hipStream_t) {
  no_device();
}
}  // namespace hss
