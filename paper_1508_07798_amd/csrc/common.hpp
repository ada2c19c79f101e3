// Shared scalar types, traits and error handling for the HSS library.
#pragma once

#include <type_traits>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#define HD __host__ __device__ __forceinline__
#else
#define HD inline
#endif

namespace hss {

// ---------------------------------------------------------------- scalars
struct cf {
  float x, y;
};
struct cd {
  double x, y;
};

HD cf operator+(cf a, cf b) { return {a.x + b.x, a.y + b.y}; }
HD cf operator-(cf a, cf b) { return {a.x - b.x, a.y - b.y}; }
HD cf operator-(cf a) { return {-a.x, -a.y}; }
HD cf operator*(cf a, cf b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
HD cf operator*(float s, cf b) { return {s * b.x, s * b.y}; }
HD cd operator+(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
HD cd operator-(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
HD cd operator-(cd a) { return {-a.x, -a.y}; }
HD cd operator*(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
HD cd operator*(double s, cd b) { return {s * b.x, s * b.y}; }

template <class T> struct traits;
template <> struct traits<float> {
  using real = float;
  using wide = double;           // FP64 counterpart
  static constexpr bool cplx = false;
  HD static float zero() { return 0.f; }
  HD static float one() { return 1.f; }
  HD static float abs2(float a) { return a * a; }
  HD static float conj(float a) { return a; }
  HD static float mk(double re, double) { return (float)re; }
  HD static float re(float a) { return a; }
  HD static float im(float) { return 0.f; }
};
template <> struct traits<double> {
  using real = double;
  using wide = double;
  static constexpr bool cplx = false;
  HD static double zero() { return 0.0; }
  HD static double one() { return 1.0; }
  HD static double abs2(double a) { return a * a; }
  HD static double conj(double a) { return a; }
  HD static double mk(double re, double) { return re; }
  HD static double re(double a) { return a; }
  HD static double im(double) { return 0.0; }
};
template <> struct traits<cf> {
  using real = float;
  using wide = cd;
  static constexpr bool cplx = true;
  HD static cf zero() { return {0.f, 0.f}; }
  HD static cf one() { return {1.f, 0.f}; }
  HD static float abs2(cf a) { return a.x * a.x + a.y * a.y; }
  HD static cf conj(cf a) { return {a.x, -a.y}; }
  HD static cf mk(double re, double im) { return {(float)re, (float)im}; }
  HD static float re(cf a) { return a.x; }
  HD static float im(cf a) { return a.y; }
};
template <> struct traits<cd> {
  using real = double;
  using wide = cd;
  static constexpr bool cplx = true;
  HD static cd zero() { return {0.0, 0.0}; }
  HD static cd one() { return {1.0, 0.0}; }
  HD static double abs2(cd a) { return a.x * a.x + a.y * a.y; }
  HD static cd conj(cd a) { return {a.x, -a.y}; }
  HD static cd mk(double re, double im) { return {re, im}; }
  HD static double re(cd a) { return a.x; }
  HD static double im(cd a) { return a.y; }
};

// scalar helpers usable for every T
HD float sc_mul(float a, float b) { return a * b; }
HD double sc_mul(double a, double b) { return a * b; }
HD cf sc_mul(cf a, cf b) { return a * b; }
HD cd sc_mul(cd a, cd b) { return a * b; }
HD float sc_inv(float a) { return 1.f / a; }
HD double sc_inv(double a) { return 1.0 / a; }
HD cf sc_inv(cf a) {
  float d = a.x * a.x + a.y * a.y;
  return {a.x / d, -a.y / d};
}
HD cd sc_inv(cd a) {
  double d = a.x * a.x + a.y * a.y;
  return {a.x / d, -a.y / d};
}
// fused a - b*c
HD float sc_fms(float a, float b, float c) { return a - b * c; }
HD double sc_fms(double a, double b, double c) { return a - b * c; }
HD cf sc_fms(cf a, cf b, cf c) { return a - b * c; }
HD cd sc_fms(cd a, cd b, cd c) { return a - b * c; }
// component-wise select (a ternary on a 16-byte struct can be lowered to a select of
// addresses through private memory)
template <class T> HD T sel(bool c, T a, T b) {
  return traits<T>::mk(c ? traits<T>::re(a) : traits<T>::re(b), c ? traits<T>::im(a) : traits<T>::im(b));
}
// conversions between precisions
HD double to_wide(float a) { return (double)a; }
HD double to_wide(double a) { return a; }
HD cd to_wide(cf a) { return {(double)a.x, (double)a.y}; }
HD cd to_wide(cd a) { return a; }
template <class T> HD T narrow(double a);
template <class T> HD T narrow(cd a);
template <> HD float narrow<float>(double a) { return (float)a; }
template <> HD double narrow<double>(double a) { return a; }
template <> HD cf narrow<cf>(cd a) { return {(float)a.x, (float)a.y}; }
template <> HD cd narrow<cd>(cd a) { return a; }

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

}  // namespace hss

#ifdef __HIPCC__
#define HIP_CHECK(expr)                                                                   \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      throw ::hss::Error(-5, std::string(#expr " failed: ") + hipGetErrorString(_e) +     \
                                 " at " + __FILE__ + ":" + std::to_string(__LINE__));     \
  } while (0)
#endif

#ifdef __HIPCC__
namespace hss {
// compile-time loop: f(std::integral_constant<int, I>) for I in [I0, N)
template <int I0, int N, class F> __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I0 < N) {
    f(std::integral_constant<int, I0>{});
    static_for<I0 + 1, N>(f);
  }
}

// ------------------------------------------------------------------ DPP reductions
// Cross-lane moves within 16-lane rows of a wave64 (gfx9 DPP encodings):
// 0xB1 = quad_perm [1,0,3,2], 0x4E = quad_perm [2,3,0,1],
// 0x141 = row_half_mirror (8 lanes), 0x140 = row_mirror (16 lanes).
// Each step pairs every lane with one partner, so after log2(width) steps all
// lanes of a group hold the same, bit-identical result (a + b == b + a).
template <int CTRL> __device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ __forceinline__ float dpp_v(float v) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL> __device__ __forceinline__ double dpp_v(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<CTRL>((int)(b & 0xffffffffll));
  const int hi = dpp_i<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float rdlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double rdlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ int rdlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// sum over aligned groups of GL (2, 4, 8, 16 or 32) lanes
template <int GL, class R> __device__ __forceinline__ R group_sum(R v) {
  static_assert(GL == 2 || GL == 4 || GL == 8 || GL == 16 || GL == 32, "group width");
  v = v + dpp_v<0xB1>(v);
  if (GL >= 4) v = v + dpp_v<0x4E>(v);
  if (GL >= 8) v = v + dpp_v<0x141>(v);
  if (GL >= 16) v = v + dpp_v<0x140>(v);
  if (GL >= 32) v = v + __shfl_xor(v, 16, 64);
  return v;
}
// sum over the whole wave, uniform result (rows combined in a fixed order)
template <class R> __device__ __forceinline__ R wave_sum(R v) {
  v = group_sum<16>(v);
  return ((rdlane(v, 0) + rdlane(v, 16)) + rdlane(v, 32)) + rdlane(v, 48);
}
// (value, index) maximum with ties to the lowest index over the whole wave; uniform
template <class R> __device__ __forceinline__ void wave_argmax(R& v, int& i) {
  auto step = [&](R v2, int i2) {
    // branch-free: the compare result selects, no exec-mask regions
    const bool take = (v2 > v) | ((v2 == v) & (i2 < i));
    v = take ? v2 : v;
    i = take ? i2 : i;
  };
  step(dpp_v<0xB1>(v), dpp_i<0xB1>(i));
  step(dpp_v<0x4E>(v), dpp_i<0x4E>(i));
  step(dpp_v<0x141>(v), dpp_i<0x141>(i));
  step(dpp_v<0x140>(v), dpp_i<0x140>(i));
  R bv = rdlane(v, 0);
  int bi = rdlane(i, 0);
  for (int r = 16; r < 64; r += 16) {
    const R v2 = rdlane(v, r);
    const int i2 = rdlane(i, r);
    if (v2 > bv || (v2 == bv && i2 < bi)) {
      bv = v2;
      bi = i2;
    }
  }
  v = bv;
  i = bi;
}
}  // namespace hss
#endif
