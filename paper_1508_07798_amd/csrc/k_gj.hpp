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

#include <type_traits>

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

// compile-time loop: f(std::integral_constant<int, I>) for I in [I0, N)
template <int I0, int N, class F> __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I0 < N) {
    f(std::integral_constant<int, I0>{});
    static_for<I0 + 1, N>(f);
  }
}

constexpr int GJ_PANEL_THREADS = 512;

// LU with partial pivoting of the panel rows j0..n-1, columns j0..j0+w-1.
// Rows are not moved: the pivot of column c is tracked as a physical row and
// every thread keeps updating the rows it owns, so one barrier per column
// suffices (the argmax partials are double buffered). The physical pivot
// sequence is turned into the usual sequence of row interchanges at the end.
// Dynamic LDS: the panel (Rr x w), w x w for Pinv and 2 Rr ints for the
// interchange bookkeeping; or global scratch when it does not fit.
template <class T, bool LDS, int NB>
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
  T* Pi = LDS ? (T*)smem_raw + (size_t)Rr * w : g.pinv;  // w x w region (LDS layout anchor)
  __shared__ R red_v[2][NW];
  __shared__ int red_i[2][NW];
  __shared__ int s_pphys[64];   // physical pivot row of each panel column
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // panel load, four independent loads in flight per thread
  for (int idx0 = tid; idx0 < Rr * w; idx0 += 4 * NT) {
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = idx0 + u * NT;
      v[u] = idx < Rr * w ? g.M[(j0 + idx % Rr) + (size_t)(j0 + idx / Rr) * g.n] : traits<T>::zero();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = idx0 + u * NT;
      if (idx < Rr * w) P[idx] = v[u];
    }
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
    wave_argmax(best, bi);
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
    // multipliers first, then the trailing columns in chunks of 16: the chunk of
    // the pivot row sits in registers and each own row's chunk is loaded, updated
    // and stored as one unrolled block (no pivot-row reload between stores)
    t = 0;
    for (int r = tid; r < Rr; r += NT, ++t) {
      if ((mine >> t) & 1ull) continue;
      P[r + (size_t)c * Rr] = sc_mul(P[r + (size_t)c * Rr], inv);
    }
    if (w == NB) {
      // full-width panel: branch-free chunks (unconditional loads, select, store back);
      // values are held as separate real / imaginary arrays so they stay in registers
      using R = typename traits<T>::real;
#pragma unroll
      for (int ch = 0; ch < NB; ch += 16) {
        if (ch + 15 <= c) continue;
        R pre[16], pim[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const T v = P[p + (size_t)(ch + u) * Rr];
          pre[u] = traits<T>::re(v);
          pim[u] = traits<T>::im(v);
        }
        t = 0;
        for (int r = tid; r < Rr; r += NT, ++t) {
          if ((mine >> t) & 1ull) continue;
          const T l = P[r + (size_t)c * Rr];
          R rre[16], rim[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const T v = P[r + (size_t)(ch + u) * Rr];
            rre[u] = traits<T>::re(v);
            rim[u] = traits<T>::im(v);
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const T rv = traits<T>::mk(rre[u], rim[u]);
            const T nv = sc_fms(rv, l, traits<T>::mk(pre[u], pim[u]));
            P[r + (size_t)(ch + u) * Rr] = (ch + u > c) ? nv : rv;
          }
        }
      }
    } else {
      // last, narrower panel
      t = 0;
      for (int r = tid; r < Rr; r += NT, ++t) {
        if ((mine >> t) & 1ull) continue;
        const T l = P[r + (size_t)c * Rr];
        for (int cc = c + 1; cc < w; ++cc)
          P[r + (size_t)cc * Rr] = sc_fms(P[r + (size_t)cc * Rr], l, P[p + (size_t)cc * Rr]);
      }
    }
  }
  __syncthreads();
  // interchange sequence (LAPACK style: row j0+c <-> row piv[j0+c], in order) from the
  // physical pivot rows; phys_at / pos_of live in the csave scratch (2 Rr ints <= n nb T)
  {
    int* phys_at = LDS ? (int*)(Pi + (size_t)w * w) : (int*)g.csave;
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
  // Pinv = U11^{-1} L11^{-1}; row c of L11 / U11 is physical row s_pphys[c]. Groups of 32
  // lanes: lane gl holds row gl of the packed L\U block in registers, a group computes
  // one column of Pinv by forward then backward substitution, broadcasting each
  // finished entry with readlane (the step index is uniform across the wave).
  __syncthreads();
  {
    const int gg = tid >> 5, gl = tid & 31, half = tid & 32;
    // complex double rows do not fit in registers next to the rest: read them per step
    constexpr bool REG = sizeof(T) <= 8;
    constexpr int NR = REG ? NB : 1;
    T row[NR];
    const int pr = gl < w ? s_pphys[gl] : 0;
    auto rowv = [&](int i) -> T {
      if (REG) return row[REG ? i : 0];
      return (gl < w && i < w) ? P[pr + (size_t)i * Rr] : traits<T>::zero();
    };
    if (REG) {
#pragma unroll
      for (int i = 0; i < NR; ++i) row[i] = (gl < w && i < w) ? P[pr + (size_t)i * Rr] : traits<T>::zero();
    }
    for (int j0c = 0; j0c < w; j0c += NT / 32) {
      const int j = j0c + gg;
      T x = (gl == j) ? traits<T>::one() : traits<T>::zero();
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const R a0 = rdlane(traits<T>::re(x), i), a1 = rdlane(traits<T>::re(x), 32 + i);
        const R b0 = rdlane(traits<T>::im(x), i), b1 = rdlane(traits<T>::im(x), 32 + i);
        const T xi = traits<T>::mk(half ? a1 : a0, half ? b1 : b0);
        if (i < w && gl > i) x = sc_fms(x, rowv(i), xi);
      }
#pragma unroll
      for (int ii = NB - 1; ii >= 0; --ii) {
        if (ii < w && gl == ii) {
          const T d = rowv(ii);
          x = traits<T>::abs2(d) == 0 ? x : sc_mul(x, sc_inv(d));
        }
        const R a0 = rdlane(traits<T>::re(x), ii), a1 = rdlane(traits<T>::re(x), 32 + ii);
        const R b0 = rdlane(traits<T>::im(x), ii), b1 = rdlane(traits<T>::im(x), 32 + ii);
        const T xi = traits<T>::mk(half ? a1 : a0, half ? b1 : b0);
        if (ii < w && gl < ii) x = sc_fms(x, rowv(ii), xi);
      }
      if (j < w && gl < w) g.pinv[gl + j * w] = x;
    }
  }
}

// Register-resident variant of the panel LU: thread tid owns rows tid + t * NT
// (t < RPT) of the panel and keeps their NB columns in registers; only the
// pivot row travels, through LDS (two barriers per column). The pivot rows are
// kept in LDS (packed L\U rows) for the pivot-block inverse. Pivots, the
// interchange sequence and Pinv are produced exactly as by gj_panel_kernel.
template <class T, int NB, int RPT>
__global__ __launch_bounds__(GJ_PANEL_THREADS) void gj_panel_reg_kernel(const GjDesc<T>* __restrict__ descs,
                                                                        int j0, int nb) {
  using R = typename traits<T>::real;
  constexpr int NT = GJ_PANEL_THREADS, NW = NT / 64;
  const GjDesc<T> g = descs[blockIdx.x];
  if (j0 >= g.n) return;
  const int w = min(nb, g.n - j0);
  const int Rr = g.n - j0;
  __shared__ R red_v[2][NW];
  __shared__ int red_i[2][NW];
  __shared__ int s_pphys[NB];
  __shared__ T s_lu[NB][NB + 1];  // packed L\U row of the pivot of column c, in order
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int* phys_at = (int*)smem_raw;  // 2 Rr ints
  int* pos_of = phys_at + Rr;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  using V = T;
  R re[RPT][NB], im[RPT][NB];
  static_for<0, RPT>([&](auto tidx) {
    constexpr int t = decltype(tidx)::value;
    const int r = tid + t * NT;
    static_for<0, NB>([&](auto ci) {
      constexpr int cc = decltype(ci)::value;
      const V v = (r < Rr && cc < w) ? g.M[(j0 + r) + (size_t)(j0 + cc) * g.n] : traits<T>::zero();
      re[t][cc] = traits<T>::re(v);
      im[t][cc] = traits<T>::im(v);
    });
  });
  unsigned done = 0;  // bit t: own row t is a pivot row
  // the column loop is expanded at compile time so that every register index is a constant
  static_for<0, NB>([&](auto cidx) {
    constexpr int c = decltype(cidx)::value;
    if (c < w) {
      R best = -1;
      int bi = 0x7fffffff;
      static_for<0, RPT>([&](auto tidx) {
        constexpr int t = decltype(tidx)::value;
        const int r = tid + t * NT;
        const R v = re[t][c] * re[t][c] + im[t][c] * im[t][c];
        if (r < Rr && !((done >> t) & 1u) && (v > best || (v == best && r < bi))) {
          best = v;
          bi = r;
        }
      });
      wave_argmax(best, bi);
      if (lane == 0) {
        red_v[c & 1][wave] = best;
        red_i[c & 1][wave] = bi;
      }
      __syncthreads();
      R bv = red_v[c & 1][0];
      int p = red_i[c & 1][0];
      for (int k = 1; k < NW; ++k) argmax_pair(bv, p, red_v[c & 1][k], red_i[c & 1][k]);
      if (p < 0 || p >= Rr) {
        // a NaN column: take the first row that is not a pivot yet
        p = Rr;
        for (int r = 0; r < Rr && p == Rr; ++r) {
          bool used = false;
          for (int q = 0; q < c; ++q) used |= (s_pphys[q] == r);
          if (!used) p = r;
        }
      }
      // the owner publishes the pivot row
      if (p % NT == tid) {
        // values picked by selects (a branch per row slot would let the compiler merge
        // the register reads into one indexed access, which forces the rows to scratch)
        const int ts = p / NT;
        done |= 1u << ts;
        static_for<0, NB>([&](auto ci) {
          constexpr int cc = decltype(ci)::value;
          R vr = re[0][cc], vi = im[0][cc];
          static_for<1, RPT>([&](auto tidx) {
            constexpr int t = decltype(tidx)::value;
            R xr = re[t][cc], xi = im[t][cc];
            asm("" : "+v"(xr), "+v"(xi));  // opaque copies: keeps the selects on values
            vr = ts == t ? xr : vr;
            vi = ts == t ? xi : vi;
          });
          s_lu[c][cc] = traits<T>::mk(vr, vi);
        });
        s_pphys[c] = p;
      }
      __syncthreads();
      const T pv = s_lu[c][c];
      const bool zero = traits<T>::abs2(pv) == 0;
      if (zero && tid == 0) *g.flag = 1;
      const T inv = zero ? traits<T>::zero() : sc_inv(pv);
      static_for<0, RPT>([&](auto tidx) {
        constexpr int t = decltype(tidx)::value;
        if (!((done >> t) & 1u)) {
          const T l = sc_mul(traits<T>::mk(re[t][c], im[t][c]), inv);
          re[t][c] = traits<T>::re(l);
          im[t][c] = traits<T>::im(l);
          static_for<c + 1, NB>([&](auto ci) {
            constexpr int cc = decltype(ci)::value;
            const T nv = sc_fms(traits<T>::mk(re[t][cc], im[t][cc]), l, s_lu[c][cc]);
            re[t][cc] = traits<T>::re(nv);
            im[t][cc] = traits<T>::im(nv);
          });
        }
      });
    }
  });
  __syncthreads();
  // interchange sequence (rows j0 + c <-> piv[j0 + c], in order)
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
  // Pinv = U11^{-1} L11^{-1} from the packed rows, 32-lane groups, readlane broadcasts
  {
    const int gg = tid >> 5, gl = tid & 31, half = tid & 32;
    for (int j0c = 0; j0c < w; j0c += NT / 32) {
      const int j = j0c + gg;
      T x = (gl == j) ? traits<T>::one() : traits<T>::zero();
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const R a0 = rdlane(traits<T>::re(x), i), a1 = rdlane(traits<T>::re(x), 32 + i);
        const R b0 = rdlane(traits<T>::im(x), i), b1 = rdlane(traits<T>::im(x), 32 + i);
        const T xi = traits<T>::mk(half ? a1 : a0, half ? b1 : b0);
        if (i < w && gl > i && gl < w) x = sc_fms(x, s_lu[gl][i], xi);
      }
#pragma unroll
      for (int ii = NB - 1; ii >= 0; --ii) {
        if (ii < w && gl == ii) {
          const T d = s_lu[ii][ii];
          x = traits<T>::abs2(d) == 0 ? x : sc_mul(x, sc_inv(d));
        }
        const R a0 = rdlane(traits<T>::re(x), ii), a1 = rdlane(traits<T>::re(x), 32 + ii);
        const R b0 = rdlane(traits<T>::im(x), ii), b1 = rdlane(traits<T>::im(x), 32 + ii);
        const T xi = traits<T>::mk(half ? a1 : a0, half ? b1 : b0);
        if (ii < w && gl < ii) x = sc_fms(x, s_lu[gl][ii], xi);
      }
      if (j < w && gl < w) g.pinv[gl + j * w] = x;
    }
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
