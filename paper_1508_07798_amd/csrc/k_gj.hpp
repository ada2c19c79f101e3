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

constexpr int GJ_PANEL_THREADS = 512;

// LU with partial pivoting of the panel rows j0..n-1, columns j0..j0+w-1.
// Rows are not moved: the pivot of column c is tracked as a physical row and
// every thread keeps updating the rows it owns, so one barrier per column
// suffices (the argmax partials are double buffered). The physical pivot
// sequence is turned into the usual sequence of row interchanges at the end.
// Dynamic LDS: the panel (Rr x w) plus w x w for Pinv, or a global scratch
// panel when it does not fit.
template <class T, bool LDS>
__global__ __launch_bounds__(GJ_PANEL_THREADS) void gj_panel_kernel(const GjDesc<T>* __restrict__ descs,
                                                                    int j0, int nb) {
  using R = typename traits<T>::real;
  constexpr int NT = GJ_PANEL_THREADS, NW = NT / 64;
  const GjDesc<T> g = descs[blockIdx.x];
  if (j0 >= g.n) return;
  const int w = min(nb, g.n - j0);
  const int Rr = g.n - j0;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* P = LDS ? (T*)smem_raw : g.gpanel;
  T* Pi = LDS ? (T*)smem_raw + (size_t)Rr * w : g.pinv;  // w x w (ld w)
  __shared__ R red_v[2][NW];
  __shared__ int red_i[2][NW];
  __shared__ int s_pphys[64];   // physical pivot row of each panel column
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int idx = tid; idx < Rr * w; idx += NT) {
    const int r = idx % Rr, c = idx / Rr;
    P[r + (size_t)c * Rr] = g.M[(j0 + r) + (size_t)(j0 + c) * g.n];
  }
  __syncthreads();
  // pivoted[r] is implied by s_pphys; each thread tracks its own rows' state in a bit mask
  // (at most Rr / NT + 1 rows per thread, <= 64 supported)
  unsigned long long mine = 0;  // bit t set: row tid + t*NT already chosen as a pivot
  for (int c = 0; c < w; ++c) {
    // partial argmax of |P(r, c)|^2 over not-yet-pivoted rows
    R best = -1;
    int bi = 0x7fffffff;
    int t = 0;
    for (int r = tid; r < Rr; r += NT, ++t) {
      if ((mine >> t) & 1ull) continue;
      const R v = traits<T>::abs2(P[r + (size_t)c * Rr]);
      argmax_pair(best, bi, v, r);
    }
    for (int off = 32; off > 0; off >>= 1) {
      const R v2 = __shfl_xor(best, off);
      const int i2 = __shfl_xor(bi, off);
      argmax_pair(best, bi, v2, i2);
    }
    if (lane == 0) {
      red_v[c & 1][wave] = best;
      red_i[c & 1][wave] = bi;
    }
    __syncthreads();
    R bv = red_v[c & 1][0];
    int p = red_i[c & 1][0];
    for (int k = 1; k < NW; ++k) argmax_pair(bv, p, red_v[c & 1][k], red_i[c & 1][k]);
    if (p < 0 || p >= Rr) {  // a NaN column leaves no candidate: take the first free row
      p = 0;
      for (int r = 0; r < Rr; ++r) {
        bool used = false;
        for (int q = 0; q < c; ++q) used |= (s_pphys[q] == r);
        if (!used) {
          p = r;
          break;
        }
      }
    }
    if (tid == 0) s_pphys[c] = p;
    if (p % NT == tid) mine |= 1ull << (p / NT);
    const T pv = P[p + (size_t)c * Rr];
    const bool zero = traits<T>::abs2(pv) == 0;
    if (zero && tid == 0) *g.flag = 1;
    const T inv = zero ? traits<T>::zero() : sc_inv(pv);
    t = 0;
    for (int r = tid; r < Rr; r += NT, ++t) {
      if ((mine >> t) & 1ull) continue;
      const T l = sc_mul(P[r + (size_t)c * Rr], inv);
      P[r + (size_t)c * Rr] = l;
      for (int cc = c + 1; cc < w; ++cc)
        P[r + (size_t)cc * Rr] = sc_fms(P[r + (size_t)cc * Rr], l, P[p + (size_t)cc * Rr]);
    }
  }
  __syncthreads();
  // interchange sequence (LAPACK style: row j0+c <-> row piv[j0+c], in order) from the
  // physical pivot rows; phys_at / pos_of live in the csave scratch (2 Rr ints <= n nb T)
  {
    int* phys_at = (int*)g.csave;
    int* pos_of = phys_at + Rr;
    for (int r = tid; r < Rr; r += NT) {
      phys_at[r] = r;
      pos_of[r] = r;
    }
    __syncthreads();
    if (tid == 0) {
      for (int c = 0; c < w; ++c) {
        const int pp = s_pphys[c];
        const int q = pos_of[pp];
        const int pc = phys_at[c];
        phys_at[c] = pp;
        phys_at[q] = pc;
        pos_of[pp] = c;
        pos_of[pc] = q;
        g.piv[j0 + c] = j0 + q;
      }
    }
  }
  // Pinv = U11^{-1} L11^{-1}; row c of L11 / U11 is physical row s_pphys[c]
  if (tid < w) {
    const int j = tid;
    for (int i = 0; i < w; ++i) {
      T y = (i == j) ? traits<T>::one() : traits<T>::zero();
      const int pi = s_pphys[i];
      for (int k = 0; k < i; ++k) y = sc_fms(y, P[pi + (size_t)k * Rr], Pi[k + j * w]);
      Pi[i + j * w] = y;
    }
    for (int i = w - 1; i >= 0; --i) {
      const int pi = s_pphys[i];
      T x = Pi[i + j * w];
      for (int k = i + 1; k < w; ++k) x = sc_fms(x, P[pi + (size_t)k * Rr], Pi[k + j * w]);
      const T d = P[pi + (size_t)i * Rr];
      Pi[i + j * w] = traits<T>::abs2(d) == 0 ? x : sc_mul(x, sc_inv(d));
    }
    if (LDS)
      for (int i = 0; i < w; ++i) g.pinv[i + j * w] = Pi[i + j * w];
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
