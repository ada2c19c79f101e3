// Batched blocked Gauss-Jordan elimination with partial pivoting.
//
// For every box of a wave, M = [A^_ii | A^_ib] (n x (n + m), column-major)
// is reduced in place to [A^_ii^{-1} | X], X = A^_ii^{-1} A^_ib: the
// elimination of I^ behind equation (32). Per panel of nb columns:
//   1. gj_panel: LU with partial pivoting of the panel rows j0..n-1 (in LDS),
//      giving the pivot rows and Pinv = (L11 U11)^{-1} of the pivot block;
//   2. gj_rows: apply the row swaps to every column, scale the pivot rows
//      R' = Pinv * M(j0:j1, :) (the panel columns become Pinv), save the
//      swapped panel columns (pivot rows zeroed) and zero them in M;
//   3. one GEMM over all rows: M -= Csave * R'.
// The elimination of the panel columns from every row (not only the rows
// below) is what turns the LU of the panel into a Gauss-Jordan step; all
// flops except the panel's sit in the GEMM. At the end the columns of the
// inverse are swapped back in reverse pivot order (gj_unswap).
#pragma once

#include "common.hpp"

namespace hss {

template <class T> struct GjDesc {
  T* M;          // n x W, ld = n
  int n, W;
  int* piv;      // [n] global pivot rows
  T* pinv;       // nb x nb scratch
  T* csave;      // n x nb scratch
  T* rbuf;       // nb x W scratch
  T* gpanel;     // (n x nb) scratch when the panel does not fit in LDS
  int* flag;     // set to 1 on an exactly zero pivot
};

template <class R> __device__ inline void argmax_pair(R& v, int& i, R v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

template <class T, bool LDS>
__global__ __launch_bounds__(256) void gj_panel_kernel(const GjDesc<T>* __restrict__ descs,
                                                       int j0, int nb) {
  using R = typename traits<T>::real;
  const GjDesc<T> g = descs[blockIdx.x];
  if (j0 >= g.n) return;
  const int w = min(nb, g.n - j0);
  const int Rr = g.n - j0;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* P = LDS ? (T*)smem_raw : g.gpanel;
  __shared__ R red_v[4];
  __shared__ int red_i[4];
  __shared__ int s_piv[64];
  __shared__ T s_inv[32 * 32];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < Rr * w; idx += 256) {
    int r = idx % Rr, c = idx / Rr;
    P[r + (size_t)c * Rr] = g.M[(j0 + r) + (size_t)(j0 + c) * g.n];
  }
  __syncthreads();
  for (int c = 0; c < w; ++c) {
    R best = -1;
    int bi = 0x7fffffff;
    for (int r = c + tid; r < Rr; r += 256) {
      R v = traits<T>::abs2(P[r + (size_t)c * Rr]);
      argmax_pair(best, bi, v, r);
    }
    for (int off = 32; off > 0; off >>= 1) {
      R v2 = __shfl_xor(best, off);
      int i2 = __shfl_xor(bi, off);
      argmax_pair(best, bi, v2, i2);
    }
    if ((tid & 63) == 0) {
      red_v[tid >> 6] = best;
      red_i[tid >> 6] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      R bv = red_v[0];
      int bidx = red_i[0];
      for (int k = 1; k < 4; ++k) argmax_pair(bv, bidx, red_v[k], red_i[k]);
      // a NaN column leaves no candidate: keep the diagonal row
      if (bidx < c || bidx >= Rr) bidx = c;
      s_piv[c] = bidx;
    }
    __syncthreads();
    const int p = s_piv[c];
    if (p != c)
      for (int cc = tid; cc < w; cc += 256) {
        T tmp = P[c + (size_t)cc * Rr];
        P[c + (size_t)cc * Rr] = P[p + (size_t)cc * Rr];
        P[p + (size_t)cc * Rr] = tmp;
      }
    __syncthreads();
    const T pv = P[c + (size_t)c * Rr];
    const bool zero = traits<T>::abs2(pv) == 0;
    if (zero && tid == 0) *g.flag = 1;
    const T inv = zero ? traits<T>::zero() : sc_inv(pv);
    for (int r = c + 1 + tid; r < Rr; r += 256) {
      T l = sc_mul(P[r + (size_t)c * Rr], inv);
      P[r + (size_t)c * Rr] = l;
      for (int cc = c + 1; cc < w; ++cc)
        P[r + (size_t)cc * Rr] = sc_fms(P[r + (size_t)cc * Rr], l, P[c + (size_t)cc * Rr]);
    }
    __syncthreads();
  }
  if (tid < w) g.piv[j0 + tid] = j0 + s_piv[tid];
  // Pinv = U11^{-1} L11^{-1}, one column per thread
  if (tid < w) {
    const int j = tid;
    for (int i = 0; i < w; ++i) {
      T y = (i == j) ? traits<T>::one() : traits<T>::zero();
      for (int k = 0; k < i; ++k) y = sc_fms(y, P[i + (size_t)k * Rr], s_inv[k + j * 32]);
      s_inv[i + j * 32] = y;
    }
    for (int i = w - 1; i >= 0; --i) {
      T x = s_inv[i + j * 32];
      for (int k = i + 1; k < w; ++k) x = sc_fms(x, P[i + (size_t)k * Rr], s_inv[k + j * 32]);
      T d = P[i + (size_t)i * Rr];
      s_inv[i + j * 32] = traits<T>::abs2(d) == 0 ? x : sc_mul(x, sc_inv(d));
    }
    for (int i = 0; i < w; ++i) g.pinv[i + j * w] = s_inv[i + j * 32];
  }
}

// Row swaps, pivot-row scaling and panel bookkeeping; grid (tiles of 64 columns, box).
template <class T>
__global__ __launch_bounds__(256) void gj_rows_kernel(const GjDesc<T>* __restrict__ descs,
                                                      int j0, int nb) {
  const GjDesc<T> g = descs[blockIdx.y];
  if (j0 >= g.n) return;
  const int w = min(nb, g.n - j0);
  const int c0 = blockIdx.x * 64;
  if (c0 >= g.W) return;
  const int cw = min(64, g.W - c0);
  __shared__ T s_pinv[32 * 32];
  __shared__ T s_seg[32][65];
  __shared__ int s_piv[32];
  const int tid = threadIdx.x;
  for (int i = tid; i < w * w; i += 256) s_pinv[i] = g.pinv[i];
  if (tid < w) s_piv[tid] = g.piv[j0 + tid];
  __syncthreads();
  // 1. swaps, column by column (sequential in the pivot order)
  if (tid < cw) {
    T* col = g.M + (size_t)(c0 + tid) * g.n;
    for (int i = 0; i < w; ++i) {
      int p = s_piv[i];
      if (p != j0 + i) {
        T a = col[j0 + i];
        col[j0 + i] = col[p];
        col[p] = a;
      }
    }
  }
  __syncthreads();
  // 2. panel columns: save (pivot rows zeroed) and clear in M
  const bool has_panel = (j0 < c0 + cw) && (j0 + w > c0);
  if (has_panel) {
    for (int idx = tid; idx < g.n * w; idx += 256) {
      int r = idx % g.n, c = idx / g.n;
      T* mp = g.M + r + (size_t)(j0 + c) * g.n;
      bool pivrow = r >= j0 && r < j0 + w;
      g.csave[r + (size_t)c * g.n] = pivrow ? traits<T>::zero() : *mp;
      if (!pivrow) *mp = traits<T>::zero();
    }
  }
  // 3. stage the pivot-row segment, then R' = Pinv * segment
  for (int idx = tid; idx < w * cw; idx += 256) {
    int i = idx % w, c = idx / w;
    s_seg[i][c] = g.M[(j0 + i) + (size_t)(c0 + c) * g.n];
  }
  __syncthreads();
  for (int idx = tid; idx < w * cw; idx += 256) {
    int i = idx % w, c = idx / w;
    int gc = c0 + c;
    T v;
    if (gc >= j0 && gc < j0 + w) {
      v = s_pinv[i + (gc - j0) * w];
    } else {
      v = traits<T>::zero();
      for (int k = 0; k < w; ++k) v = v + sc_mul(s_pinv[i + k * w], s_seg[k][c]);
    }
    g.rbuf[i + (size_t)gc * w] = v;
    g.M[(j0 + i) + (size_t)gc * g.n] = v;
  }
}

// Undo the row interchanges on the columns of the inverse: for j = n-1..0
// swap columns j and piv[j]. Each thread owns rows, so no synchronisation.
template <class T>
__global__ __launch_bounds__(256) void gj_unswap_kernel(const GjDesc<T>* __restrict__ descs) {
  const GjDesc<T> g = descs[blockIdx.y];
  for (int r = blockIdx.x * 256 + threadIdx.x; r < g.n; r += gridDim.x * 256) {
    for (int j = g.n - 1; j >= 0; --j) {
      int p = g.piv[j];
      if (p != j) {
        T a = g.M[r + (size_t)j * g.n];
        g.M[r + (size_t)j * g.n] = g.M[r + (size_t)p * g.n];
        g.M[r + (size_t)p * g.n] = a;
      }
    }
  }
}

}  // namespace hss
