// Batched variable-size GEMM on CDNA4 matrix cores:
//   C_b = alpha * A_b * B_b + beta * C_b   (all column-major, no transposes;
//   beta is taken as 0 on an optional column window of each entry)
// for every entry b of a descriptor array, one launch for all entries.
//
// Tiles of 64 x 64 outputs per 256-thread workgroup (4 wavefronts, each a
// 32 x 32 quadrant made of 2 x 2 MFMA 16x16 blocks), or 128 x 128 for large
// real FP32 products (each wave 4 x 4 blocks). K advances in slabs of
// BK, staged through LDS with the next slab prefetched into registers while
// the current one is consumed. FP32 uses v_mfma_f32_16x16x4_f32, FP64 uses
// v_mfma_f64_16x16x4_f64; complex operands use four real products
// (re*re - im*im, re*im + im*re) on split real/imaginary LDS planes.
// Workgroups map to (entry, tile) through a prefix sum of tile counts.
#pragma once

#include "common.hpp"

namespace hss {

struct GemmDesc {
  const void* A;
  const void* B;
  void* C;
  int M, N, K;
  int lda, ldb, ldc;
  int z0, z1;  // columns [z0, z1) of C are written with beta = 0 (old values ignored)
};

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <class R> struct mfma_acc;
// Result layout of the 16x16x4 MFMA: lane l holds column l % 16; value v of the
// lane is row 4 * (l / 16) + v for FP32 and row (l / 16) + 4 * v for FP64 (both
// checked by a lane-layout probe on gfx950). Operands: lane l holds A(l % 16, l / 16)
// and B(l / 16, l % 16).
template <> struct mfma_acc<float> {
  using type = v4f;
  __device__ static inline int row(int lk, int v) { return lk * 4 + v; }
  __device__ static inline v4f mac(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct mfma_acc<double> {
  using type = v4d;
  __device__ static inline int row(int lk, int v) { return lk + 4 * v; }
  __device__ static inline v4d mac(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <class T> __device__ inline void split(T v, typename traits<T>::real& re,
                                                typename traits<T>::real& im) {
  re = traits<T>::re(v);
  im = traits<T>::im(v);
}

constexpr int GBM = 64, GBN = 64;

template <class T> struct gemm_cfg {
  // K slab per LDS stage: 16 real or complex64 values, 8 complex128 values
  static constexpr int BK = traits<T>::cplx && sizeof(T) >= 16 ? 8 : 16;
};

// Role of a GEMM launch; it only separates the kernel symbols so that a profile
// tells the Schur update, the Gauss-Jordan trailing update and the sampling apart.
enum GemmRole { GEMM_GENERIC = 0, GEMM_SCHUR = 1, GEMM_GJ_UPDATE = 2, GEMM_SAMPLE = 3 };

// One (32 WI) x (32 WI) tile of C per workgroup: the four waves in a 2 x 2 grid,
// each owning WI x WI MFMA 16x16 blocks. WI = 2 (64 x 64 tiles) serves every
// launch; WI = 4 (128 x 128 tiles) the large real FP32 products, where each
// staged value then serves twice as many outputs. (For complex64 that tile needs
// 424 registers, one wave per SIMD, and measured slower at every size.)
template <class T, int WI>
__device__ __forceinline__ void gemm_tile(const GemmDesc* __restrict__ descs, const int* __restrict__ tprefix,
                                          int nent, T alpha, T beta) {
  using R = typename traits<T>::real;
  using Acc = typename mfma_acc<R>::type;
  constexpr bool CX = traits<T>::cplx;
  // complex64 operands: planes re, im and re + im, and three real products per
  // complex one (ar br, ai bi, (ar + ai)(br + bi); Re = t0 - t1, Im = t2 - t0 - t1),
  // measured 10% faster than four on deep products. complex128: planes re, im and
  // four products (the third plane's staging cost more than the product saved).
  constexpr bool G3 = CX && std::is_same<R, float>::value;
  constexpr int NP = CX ? (G3 ? 3 : 2) : 1;
  constexpr int BK = gemm_cfg<T>::BK;
  constexpr int TM = 32 * WI, TN = 32 * WI, WT = 16 * WI;  // tile, wave tile
  constexpr int LDA_S = TM + 4, LDB_S = TN + 4;
  __shared__ R As[NP][BK][LDA_S];
  __shared__ R Bs[NP][BK][LDB_S];

  // locate the entry of this workgroup
  const int bid = blockIdx.x;
  int lo = 0, hi = nent;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (tprefix[mid] <= bid) lo = mid; else hi = mid;
  }
  const GemmDesc g = descs[lo];
  const int t = bid - tprefix[lo];
  const int tmc = (g.M + TM - 1) / TM;
  const int m0 = (t % tmc) * TM, n0 = (t / tmc) * TN;
  const T* __restrict__ Ag = (const T*)g.A;
  const T* __restrict__ Bg = (const T*)g.B;
  T* __restrict__ Cg = (T*)g.C;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * WT, wn = (wave >> 1) * WT;
  const int li = lane & 15, lk = lane >> 4;

  Acc acc[NP][WI][WI];
  for (int p = 0; p < NP; ++p)
    for (int i = 0; i < WI; ++i)
      for (int j = 0; j < WI; ++j) acc[p][i][j] = Acc{0, 0, 0, 0};

  // global -> register staging: A slab TM x BK, B slab BK x TN
  constexpr int AE = TM * BK / 256;  // elements per thread
  constexpr int BE = BK * TN / 256;
  T ra[AE], rb[BE];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      int idx = tid + e * 256;
      int i = idx % TM, k = idx / TM;
      int gi = m0 + i, gk = k0 + k;
      ra[e] = (gi < g.M && gk < g.K) ? Ag[gi + (size_t)gk * g.lda] : traits<T>::zero();
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      int idx = tid + e * 256;
      int k = idx % BK, j = idx / BK;
      int gk = k0 + k, gj = n0 + j;
      rb[e] = (gk < g.K && gj < g.N) ? Bg[gk + (size_t)gj * g.ldb] : traits<T>::zero();
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      int idx = tid + e * 256;
      int i = idx % TM, k = idx / TM;
      R re, im;
      split(ra[e], re, im);
      As[0][k][i] = re;
      if constexpr (CX) As[1][k][i] = im;
      if constexpr (G3) As[2][k][i] = re + im;
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      int idx = tid + e * 256;
      int k = idx % BK, j = idx / BK;
      R re, im;
      split(rb[e], re, im);
      Bs[0][k][j] = re;
      if constexpr (CX) Bs[1][k][j] = im;
      if constexpr (G3) Bs[2][k][j] = re + im;
    }
  };

  load(0);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    store();
    __syncthreads();
    if (k0 + BK < g.K) load(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + lk;
      R a[NP][WI], b[NP][WI];
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int i = 0; i < WI; ++i) {
          a[p][i] = As[p][kk][wm + 16 * i + li];
          b[p][i] = Bs[p][kk][wn + 16 * i + li];
        }
#pragma unroll
      for (int i = 0; i < WI; ++i)
#pragma unroll
        for (int j = 0; j < WI; ++j) {
          if constexpr (G3) {
            acc[0][i][j] = mfma_acc<R>::mac(a[0][i], b[0][j], acc[0][i][j]);
            acc[1][i][j] = mfma_acc<R>::mac(a[1][i], b[1][j], acc[1][i][j]);
            acc[2][i][j] = mfma_acc<R>::mac(a[2][i], b[2][j], acc[2][i][j]);
          } else if constexpr (CX) {
            acc[0][i][j] = mfma_acc<R>::mac(a[0][i], b[0][j], acc[0][i][j]);
            acc[0][i][j] = mfma_acc<R>::mac(-a[1][i], b[1][j], acc[0][i][j]);
            acc[1][i][j] = mfma_acc<R>::mac(a[0][i], b[1][j], acc[1][i][j]);
            acc[1][i][j] = mfma_acc<R>::mac(a[1][i], b[0][j], acc[1][i][j]);
          } else {
            acc[0][i][j] = mfma_acc<R>::mac(a[0][i], b[0][j], acc[0][i][j]);
          }
        }
    }
    __syncthreads();
  }

  // epilogue: lane holds column lane%16 and four rows of each 16x16 block. Per
  // group of RG rows of blocks (all of them for 64 x 64 tiles, one for 128 x 128,
  // which bounds the registers held), all reads of C are issued before the first
  // store (the stores could alias the reads as far as the compiler knows, which
  // would serialize read-store pairs).
  constexpr int RG = WI <= 2 ? WI : 1;
  const bool rdc = !(traits<T>::re(beta) == 0 && traits<T>::im(beta) == 0);
  static_for<0, WI / RG>([&](auto gg) {
    constexpr int i0 = decltype(gg)::value * RG;
    R cre[RG][WI][4], cim[RG][WI][4];
    static_for<0, RG>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      static_for<0, WI>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        const int col = n0 + wn + j * 16 + li;
        const bool keep = col < g.N && (col < g.z0 || col >= g.z1) && rdc;
        static_for<0, 4>([&](auto vv) {
          constexpr int v = decltype(vv)::value;
          const int row = m0 + wm + (i0 + i) * 16 + mfma_acc<R>::row(lk, v);
          const T c = (keep && row < g.M) ? Cg[row + (size_t)col * g.ldc] : traits<T>::zero();
          cre[i][j][v] = traits<T>::re(c);
          cim[i][j][v] = traits<T>::im(c);
        });
      });
    });
    static_for<0, RG>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      static_for<0, WI>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        const int col = n0 + wn + j * 16 + li;
        static_for<0, 4>([&](auto vv) {
          constexpr int v = decltype(vv)::value;
          const int row = m0 + wm + (i0 + i) * 16 + mfma_acc<R>::row(lk, v);
          if (col < g.N && row < g.M) {
            T val;
            if constexpr (G3) {
              const R t0 = acc[0][i0 + i][j][v], t1 = acc[1][i0 + i][j][v];
              val = traits<T>::mk(t0 - t1, acc[2][i0 + i][j][v] - t0 - t1);
            } else if constexpr (CX) {
              val = traits<T>::mk(acc[0][i0 + i][j][v], acc[1][i0 + i][j][v]);
            } else {
              val = acc[0][i0 + i][j][v];
            }
            Cg[row + (size_t)col * g.ldc] =
                sc_mul(alpha, val) + sc_mul(beta, traits<T>::mk(cre[i][j][v], cim[i][j][v]));
          }
        });
      });
    });
  });
}

// 64 x 64 tiles (GBM x GBN)
template <class T, int ROLE>
__global__ __launch_bounds__(256) void gemm_nn_kernel(const GemmDesc* __restrict__ descs,
                                                      const int* __restrict__ tprefix, int nent, T alpha, T beta) {
  gemm_tile<T, 2>(descs, tprefix, nent, alpha, beta);
}

// 128 x 128 tiles (GBM_BIG x GBN_BIG)
constexpr int GBM_BIG = 128, GBN_BIG = 128;
template <class T, int ROLE>
__global__ __launch_bounds__(256) void gemm_big_kernel(const GemmDesc* __restrict__ descs,
                                                       const int* __restrict__ tprefix, int nent, T alpha, T beta) {
  gemm_tile<T, 4>(descs, tprefix, nent, alpha, beta);
}

// ---------------------------------------------------------------- BF16 x 3
// Real FP32 operands on BF16 matrix cores with FP32 accumulation: every value is
// split x = hi + lo with hi = bf16(x) and lo = bf16(x - hi), and the product is
// taken as hi*hi + hi*lo + lo*hi (the lo*lo term, ~2^-16 relative, is dropped),
// which keeps about 16 significant bits, i.e. ~1e-5 relative error per product
// sum instead of BF16's ~4e-3. v_mfma_f32_16x16x32_bf16: lane l holds A(l % 16,
// 8 (l / 16) + j) and B(8 (l / 16) + j, l % 16) for j < 8; the result layout is
// that of the FP32 16x16 MFMA. Tiles, slabs and the prologue as gemm_nn_kernel.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int ROLE>
__global__ __launch_bounds__(256) void gemm_bf16x3_kernel(const GemmDesc* __restrict__ descs,
                                                          const int* __restrict__ tprefix, int nent, float alpha,
                                                          float beta) {
  constexpr int BK = 32, LDK = BK + 8;  // row pitch 80 bytes: 16-byte aligned 8-element reads
  __shared__ __attribute__((aligned(16))) __bf16 As[2][GBM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][GBN][LDK];
  const int bid = blockIdx.x;
  int lo = 0, hi = nent;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (tprefix[mid] <= bid) lo = mid; else hi = mid;
  }
  const GemmDesc g = descs[lo];
  const int t = bid - tprefix[lo];
  const int tmc = (g.M + GBM - 1) / GBM;
  const int m0 = (t % tmc) * GBM, n0 = (t / tmc) * GBN;
  const float* __restrict__ Ag = (const float*)g.A;
  const float* __restrict__ Bg = (const float*)g.B;
  float* __restrict__ Cg = (float*)g.C;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0, 0, 0, 0};
  constexpr int E = GBM * BK / 256;  // 8 values of A and of B per thread and slab
  float ra[E], rb[E];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = tid + e * 256;
      const int i = idx % GBM, k = idx / GBM;  // A: m fastest (coalesced)
      const int gi = m0 + i, gk = k0 + k;
      ra[e] = (gi < g.M && gk < g.K) ? Ag[gi + (size_t)gk * g.lda] : 0.f;
      const int kb = idx % BK, j = idx / BK;    // B: k fastest (coalesced)
      const int gkb = k0 + kb, gj = n0 + j;
      rb[e] = (gkb < g.K && gj < g.N) ? Bg[gkb + (size_t)gj * g.ldb] : 0.f;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = tid + e * 256;
      const int i = idx % GBM, k = idx / GBM;
      const __bf16 ah = (__bf16)ra[e];
      As[0][i][k] = ah;
      As[1][i][k] = (__bf16)(ra[e] - (float)ah);
      const int kb = idx % BK, j = idx / BK;
      const __bf16 bh = (__bf16)rb[e];
      Bs[0][j][kb] = bh;
      Bs[1][j][kb] = (__bf16)(rb[e] - (float)bh);
    }
  };
  load(0);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    store();
    __syncthreads();
    if (k0 + BK < g.K) load(k0 + BK);
    bf16x8 a[2][2], b[2][2];  // [plane][block]
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[p][i] = *(const bf16x8*)&As[p][wm + i * 16 + li][lk * 8];
        b[p][i] = *(const bf16x8*)&Bs[p][wn + i * 16 + li][lk * 8];
      }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], acc[i][j], 0, 0, 0);
      }
    __syncthreads();
  }
  // all reads of C before the first store (see gemm_nn_kernel)
  float cv[2][2][4];
  static_for<0, 2>([&](auto ii) {
    static_for<0, 2>([&](auto jj) {
      constexpr int i = decltype(ii)::value, j = decltype(jj)::value;
      const int col = n0 + wn + j * 16 + li;
      const bool keep = col < g.N && (col < g.z0 || col >= g.z1) && beta != 0.f;
      static_for<0, 4>([&](auto vv) {
        constexpr int v = decltype(vv)::value;
        const int row = m0 + wm + i * 16 + mfma_acc<float>::row(lk, v);
        cv[i][j][v] = (keep && row < g.M) ? Cg[row + (size_t)col * g.ldc] : 0.f;
      });
    });
  });
  static_for<0, 2>([&](auto ii) {
    static_for<0, 2>([&](auto jj) {
      constexpr int i = decltype(ii)::value, j = decltype(jj)::value;
      const int col = n0 + wn + j * 16 + li;
      static_for<0, 4>([&](auto vv) {
        constexpr int v = decltype(vv)::value;
        const int row = m0 + wm + i * 16 + mfma_acc<float>::row(lk, v);
        if (col < g.N && row < g.M) Cg[row + (size_t)col * g.ldc] = alpha * acc[i][j][v] + beta * cv[i][j][v];
      });
    });
  });
}

// Complex64 operands on BF16 matrix cores, the same three-term split per real
// product: Re C += Ar Br + (-Ai) Bi, Im C += Ar Bi + Ai Br, each real product as
// hi*hi + hi*lo + lo*hi, i.e. 12 bf16 MFMAs per 16 x 16 x 32 block. A keeps six
// bf16 planes in LDS (re, im and -im, each hi and lo; the negation is exact), B
// four. Tiles, slabs and the prologue as gemm_bf16x3_kernel.
template <int ROLE>
__global__ __launch_bounds__(256) void gemm_cbf16x3_kernel(const GemmDesc* __restrict__ descs,
                                                           const int* __restrict__ tprefix, int nent, cf alpha,
                                                           cf beta) {
  constexpr int BK = 32, LDK = BK + 8;
  __shared__ __attribute__((aligned(16))) __bf16 As[6][GBM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[4][GBN][LDK];
  const int bid = blockIdx.x;
  int lo = 0, hi = nent;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (tprefix[mid] <= bid) lo = mid; else hi = mid;
  }
  const GemmDesc g = descs[lo];
  const int t = bid - tprefix[lo];
  const int tmc = (g.M + GBM - 1) / GBM;
  const int m0 = (t % tmc) * GBM, n0 = (t / tmc) * GBN;
  const cf* __restrict__ Ag = (const cf*)g.A;
  const cf* __restrict__ Bg = (const cf*)g.B;
  cf* __restrict__ Cg = (cf*)g.C;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  v4f accr[2][2], acci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) accr[i][j] = acci[i][j] = v4f{0, 0, 0, 0};
  constexpr int E = GBM * BK / 256;  // 8 values of A and of B per thread and slab
  cf ra[E], rb[E];
  const cf z = traits<cf>::zero();
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = tid + e * 256;
      const int i = idx % GBM, k = idx / GBM;  // A: m fastest (coalesced)
      const int gi = m0 + i, gk = k0 + k;
      ra[e] = (gi < g.M && gk < g.K) ? Ag[gi + (size_t)gk * g.lda] : z;
      const int kb = idx % BK, j = idx / BK;    // B: k fastest (coalesced)
      const int gkb = k0 + kb, gj = n0 + j;
      rb[e] = (gkb < g.K && gj < g.N) ? Bg[gkb + (size_t)gj * g.ldb] : z;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = tid + e * 256;
      const int i = idx % GBM, k = idx / GBM;
      const __bf16 rh = (__bf16)ra[e].x, ih = (__bf16)ra[e].y;
      const __bf16 rl = (__bf16)(ra[e].x - (float)rh), il = (__bf16)(ra[e].y - (float)ih);
      As[0][i][k] = rh;
      As[1][i][k] = rl;
      As[2][i][k] = ih;
      As[3][i][k] = il;
      As[4][i][k] = -ih;
      As[5][i][k] = -il;
      const int kb = idx % BK, j = idx / BK;
      const __bf16 brh = (__bf16)rb[e].x, bih = (__bf16)rb[e].y;
      Bs[0][j][kb] = brh;
      Bs[1][j][kb] = (__bf16)(rb[e].x - (float)brh);
      Bs[2][j][kb] = bih;
      Bs[3][j][kb] = (__bf16)(rb[e].y - (float)bih);
    }
  };
  load(0);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    store();
    __syncthreads();
    if (k0 + BK < g.K) load(k0 + BK);
    bf16x8 a[6][2], b[4][2];  // [plane][block]
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int p = 0; p < 6; ++p) a[p][i] = *(const bf16x8*)&As[p][wm + i * 16 + li][lk * 8];
#pragma unroll
      for (int p = 0; p < 4; ++p) b[p][i] = *(const bf16x8*)&Bs[p][wn + i * 16 + li][lk * 8];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        v4f r = accr[i][j], m = acci[i][j];
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[5][i], b[2][j], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[4][i], b[3][j], r, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[4][i], b[2][j], r, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[2][j], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[3][j], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[2][j], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[3][i], b[0][j], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2][i], b[1][j], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2][i], b[0][j], m, 0, 0, 0);
        accr[i][j] = r;
        acci[i][j] = m;
      }
    __syncthreads();
  }
  // all reads of C before the first store (see gemm_nn_kernel)
  const bool rdc = !(beta.x == 0.f && beta.y == 0.f);
  cf cv[2][2][4];
  static_for<0, 2>([&](auto ii) {
    static_for<0, 2>([&](auto jj) {
      constexpr int i = decltype(ii)::value, j = decltype(jj)::value;
      const int col = n0 + wn + j * 16 + li;
      const bool keep = col < g.N && (col < g.z0 || col >= g.z1) && rdc;
      static_for<0, 4>([&](auto vv) {
        constexpr int v = decltype(vv)::value;
        const int row = m0 + wm + i * 16 + mfma_acc<float>::row(lk, v);
        cv[i][j][v] = (keep && row < g.M) ? Cg[row + (size_t)col * g.ldc] : z;
      });
    });
  });
  static_for<0, 2>([&](auto ii) {
    static_for<0, 2>([&](auto jj) {
      constexpr int i = decltype(ii)::value, j = decltype(jj)::value;
      const int col = n0 + wn + j * 16 + li;
      static_for<0, 4>([&](auto vv) {
        constexpr int v = decltype(vv)::value;
        const int row = m0 + wm + i * 16 + mfma_acc<float>::row(lk, v);
        if (col < g.N && row < g.M)
          Cg[row + (size_t)col * g.ldc] =
              sc_mul(alpha, traits<cf>::mk(accr[i][j][v], acci[i][j][v])) + sc_mul(beta, cv[i][j][v]);
      });
    });
  });
}

}  // namespace hss
