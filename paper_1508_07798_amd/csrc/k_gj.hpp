// Batched blocked Gauss-Jordan elimination with partial pivoting.
//
// For every box of a wave, M = [A^_ii | A^_ib] (n x (n + m), column-major)
// is reduced in place to [(P A^_ii)^{-1} | X], X = A^_ii^{-1} A^_ib: the
// elimination of I^ behind equation (32). P is the row permutation chosen by
// partial pivoting, recorded as rowperm ((P A)(i, :) = A(rowperm[i], :)). The
// inverse stays in that pivoted column order: A^{-1} y = (P A)^{-1} (P y), so a
// product with A^{-1} gathers its input through rowperm. Per panel of nb columns:
//   1. gj_panel: LU with partial pivoting of the panel rows j0..n-1, giving the
//      pivot rows, their net movement (at most 2 nb rows move) and
//      Pinv = (L11 U11)^{-1} of the pivot block;
//   2. gj_rows: apply the row movement to every column, form the scaled
//      pivot rows R' = Pinv * M(j0:j1, :) (Pinv in the panel columns) and the
//      saved panel columns Csave of the interchanged M (pivot block -I);
//   3. one GEMM over all rows: M = M - Csave * R', with M's old panel columns
//      ignored (beta = 0 there), which leaves R' in the pivot rows.
// The elimination of the panel columns from every row (not only the rows
// below) is what turns the LU of the panel into a Gauss-Jordan step; all
// flops except the panel's sit in the GEMM.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace hss {

template <class T> struct GjDesc {
  T* M;          // rows x W, ld = rows
  int n, W;      // n pivot columns (0 .. n-1); their pivot rows are poff .. poff + n - 1
  int rows, poff;
  T* pinv;       // nb x nb scratch
  T* csave;      // rows x nb scratch
  T* rbuf;       // nb x W scratch (wo x W for a block)
  T* gpanel;     // (rows x nb) scratch when the panel does not fit in LDS
  int* flag;     // set to 1 on an exactly zero pivot
  int* mv;       // [1 + 4 max(nb, wo)] net row movement of the current panel or block:
                 // count, then (dst, src) pairs
  int* rowperm;  // [rows] net row permutation: original row now at each position
  // second-level blocking: copy of the current block of wo columns (rows x wo)
  // and the row permutation of its elimination
  T* pb;
  int* rp_in;
};

template <class R> struct RedPair {
  R v;
  int i;
};

template <class R> __device__ inline void argmax_pair(R& v, int& i, R v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}


constexpr int GJ_PANEL_THREADS = 512;

// Net row movement of a panel, computed by one wave once the pivots of all w (<= 32)
// columns are known: position c takes its pivot row pphys[c]; the rows r0 < w that
// are not pivots fill, in increasing order, the positions >= w whose rows became
// pivots (every such pairing is a valid partial-pivoting order). Writes
// mv = [count, (dst, src), ...] with positions relative to the panel start.
// With rowperm set (wave 0 only, after rowperm's initialisation is visible), the
// same moves are applied to the row permutation: all of this wave's loads precede
// its stores, so cycles of moves need no staging.
__device__ __forceinline__ void panel_moves(int* mv, const int* pphys, int w, int* rowperm = nullptr,
                                            int base = 0) {
  const int lane = threadIdx.x & 63;
  const int pc = lane < w ? pphys[lane] : -1;
  unsigned pivlow = 0;  // bit r0: row r0 < w is a pivot
  for (int r0 = 0; r0 < w; ++r0)
    if (__ballot(pc == r0)) pivlow |= 1u << r0;
  const bool disp = lane < w && !((pivlow >> lane) & 1u);  // row `lane` leaves the pivot block
  const bool vac = lane < w && pc >= w;                     // position pc loses its row
  const bool mov = lane < w && pc != lane;
  const unsigned long long below = (1ull << lane) - 1;
  const unsigned long long bd = __ballot(disp), bv = __ballot(vac), bm = __ballot(mov);
  const int kd = __popcll(bd & below), km = __popcll(bm & below), n1 = __popcll(bm);
  int dst = -1;
  unsigned long long rem = bv;
  for (int k = 0; rem; ++k) {
    const int lv = __ffsll((long long)rem) - 1;  // uniform: k-th vacated position's lane
    rem &= rem - 1;
    const int pos = __builtin_amdgcn_readlane(pc, lv);
    if (disp && kd == k) dst = pos;
  }
  if (mov) {
    mv[1 + 2 * km] = lane;
    mv[2 + 2 * km] = pc;
  }
  if (disp) {
    mv[1 + 2 * (n1 + kd)] = dst;
    mv[2 + 2 * (n1 + kd)] = lane;
  }
  if (lane == 0) mv[0] = n1 + __popcll(bd);
  if (rowperm) {
    const int v1 = mov ? rowperm[base + pc] : 0;
    const int v2 = disp ? rowperm[base + lane] : 0;
    if (mov) rowperm[base + lane] = v1;
    if (disp) rowperm[base + dst] = v2;
  }
}

// Pinv = (L11 U11)^{-1} from the packed L\U rows of the pivot block in LDS
// (lu[c * LD + i]: row c, unit lower part left of the diagonal). Groups of 32
// lanes; lane gl works on row gl and each group solves for one column of Pinv
// (forward, then backward substitution), broadcasting every finished entry with
// readlane. Row entries are read from LDS in batches of 8. A zero diagonal entry
// leaves its row unscaled (the zero pivot is reported through the flag).
template <class T, int NB, int LD, int NT = GJ_PANEL_THREADS>
__device__ __forceinline__ void pivot_block_inverse(const T* lu, int w, T* __restrict__ pinv) {
  using R = typename traits<T>::real;
  const int tid = threadIdx.x, gg = tid >> 5, gl = tid & 31, half = tid & 32;
  const T* row = lu + (gl < w ? gl : 0) * LD;
  T dinv = traits<T>::one();
  if (gl < w) {
    const T d = row[gl];
    if (traits<T>::abs2(d) != 0) dinv = sc_inv(d);
  }
  auto bcast = [&](const T& x, int i) {
    const R a0 = rdlane(traits<T>::re(x), i), a1 = rdlane(traits<T>::re(x), 32 + i);
    const R b0 = rdlane(traits<T>::im(x), i), b1 = rdlane(traits<T>::im(x), 32 + i);
    return traits<T>::mk(half ? a1 : a0, half ? b1 : b0);
  };
  for (int j0c = 0; j0c < w; j0c += NT / 32) {
    const int j = j0c + gg;
    T x = sel(gl == j, traits<T>::one(), traits<T>::zero());
    static_for<0, NB / 8>([&](auto chi) {
      constexpr int cb = decltype(chi)::value * 8;
      if (cb < w) {
        R rr[8], ri[8];
        static_for<0, 8>([&](auto ui) {
          constexpr int u = decltype(ui)::value;
          const T v = row[cb + u];
          rr[u] = traits<T>::re(v);
          ri[u] = traits<T>::im(v);
        });
        static_for<0, 8>([&](auto ui) {
          constexpr int u = decltype(ui)::value;
          constexpr int i = cb + u;
          if (i < w) {
            const T xi = bcast(x, i);
            const T nx = sc_fms(x, traits<T>::mk(rr[u], ri[u]), xi);
            x = sel(gl > i && gl < w, nx, x);
          }
        });
      }
    });
    static_for<0, NB / 8>([&](auto chk) {
      constexpr int cb = NB - 8 - decltype(chk)::value * 8;
      if (cb < w) {
        R rr[8], ri[8];
        static_for<0, 8>([&](auto ui) {
          constexpr int u = decltype(ui)::value;
          const T v = row[cb + u];
          rr[u] = traits<T>::re(v);
          ri[u] = traits<T>::im(v);
        });
        static_for<0, 8>([&](auto ui) {
          constexpr int u = 7 - decltype(ui)::value;
          constexpr int i = cb + u;
          if (i < w) {
            x = sel(gl == i, sc_mul(x, dinv), x);
            const T xi = bcast(x, i);
            const T nx = sc_fms(x, traits<T>::mk(rr[u], ri[u]), xi);
            x = sel(gl < i, nx, x);
          }
        });
      }
    });
    if (j < w && gl < w) pinv[gl + j * w] = x;
  }
}

// LU with partial pivoting of the panel rows j0..n-1, columns j0..j0+w-1, for
// panels too tall for the register-resident kernel below. Rows are not moved:
// the pivot of column c is tracked as a physical row and every thread keeps
// updating the rows it owns, so one barrier per column suffices (the argmax
// partials are double buffered). The panel (Rr x w) sits in dynamic LDS, or in
// global scratch when it does not fit.
template <class T, bool LDS, int NB>
__global__ __launch_bounds__(GJ_PANEL_THREADS) void gj_panel_kernel(const GjDesc<T>* __restrict__ descs,
                                                                    int j0, int nb) {
  using R = typename traits<T>::real;
  constexpr int NT = GJ_PANEL_THREADS, NW = NT / 64;
  const GjDesc<T> g = descs[blockIdx.x];
  if (j0 >= g.n) return;
  const int w = min(nb, g.n - j0);
  const int base = g.poff + j0;  // first candidate row
  const int Rr = g.rows - base;  // candidate rows
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* P = LDS ? (T*)smem_raw : g.gpanel;
  __shared__ R red_v[2][NW];
  __shared__ int red_i[2][NW];
  __shared__ int s_pphys[64];     // physical pivot row of each panel column
  __shared__ T s_lu[NB][NB + 1];  // packed L\U row of the pivot of column c
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // panel load, four independent loads in flight per thread; the index of a load
  // past the panel is clamped to its first element (sel evaluates both operands)
  for (int idx0 = tid; idx0 < Rr * w; idx0 += 4 * NT) {
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = idx0 + u * NT;
      const int ic = idx < Rr * w ? idx : 0;
      v[u] = sel(idx < Rr * w, g.M[(base + ic % Rr) + (size_t)(j0 + ic / Rr) * g.rows], traits<T>::zero());
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
    // the pivot row is final from here on (multipliers left of c, U from c)
    if (tid < w) s_lu[c][tid] = P[p + (size_t)tid * Rr];
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
            P[r + (size_t)(ch + u) * Rr] = sel(ch + u > c, nv, rv);
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
  if (wave == 0) panel_moves(g.mv, s_pphys, w);
  pivot_block_inverse<T, NB, NB + 1>(&s_lu[0][0], w, g.pinv);
}

// Register-resident panel LU: thread tid owns rows tid + t * NT (t < RPT) of the
// panel and keeps their NB columns in registers; only candidate pivot rows travel,
// through LDS. The pivot rows are kept in LDS (packed L\U rows) for the pivot-block
// inverse. Pivots, row movement and Pinv are the same as from gj_panel_kernel.
template <class T, int NB, int RPT>
__global__ __launch_bounds__(GJ_PANEL_THREADS) void gj_panel_reg_kernel(const GjDesc<T>* __restrict__ descs,
                                                                        int j0, int nb) {
  using R = typename traits<T>::real;
  constexpr int NT = GJ_PANEL_THREADS, NW = NT / 64;
  const GjDesc<T> g = descs[blockIdx.x];
  if (j0 >= g.n) return;
  const int w = min(nb, g.n - j0);
  const int base = g.poff + j0;  // first candidate row
  const int Rr = g.rows - base;  // candidate rows
  __shared__ RedPair<R> s_red[2][NW];
  __shared__ int s_pphys[NB];
  __shared__ T s_lu[NB][NB + 1];  // packed L\U row of the pivot of column c, in order
  __shared__ T s_cand[2][NW][RPT][NB];  // candidate pivot row of every wave, double buffered
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  using V = T;
  R re[RPT][NB], im[RPT][NB];
  static_for<0, RPT>([&](auto tidx) {
    constexpr int t = decltype(tidx)::value;
    const int r = tid + t * NT;
    static_for<0, NB>([&](auto ci) {
      constexpr int cc = decltype(ci)::value;
      const V v = (r < Rr && cc < w) ? g.M[(base + r) + (size_t)(j0 + cc) * g.rows] : traits<T>::zero();
      re[t][cc] = traits<T>::re(v);
      im[t][cc] = traits<T>::im(v);
    });
  });
  unsigned done = 0;  // bit t: own row t is a pivot row
  // Values of the current column of the own rows; refreshed while column c is updated.
  R cr[RPT], ci[RPT];
  static_for<0, RPT>([&](auto tidx) {
    constexpr int t = decltype(tidx)::value;
    cr[t] = re[t][0];
    ci[t] = im[t][0];
  });
  // The column loop runs at run time (compact code); register indices stay
  // compile-time constants and the columns at or left of c are skipped with branches
  // on the uniform c. One barrier per column: before it, every wave publishes its best
  // candidate row (double-buffered), after it every thread reduces the wave partials
  // and reads the winning row.
  for (int c = 0; c < w; ++c) {
    const int buf = c & 1;
    R best = -1;
    int bi = 0x7fffffff;
    static_for<0, RPT>([&](auto tidx) {
      constexpr int t = decltype(tidx)::value;
      const int r = tid + t * NT;
      const R v = cr[t] * cr[t] + ci[t] * ci[t];
      const bool take = (r < Rr) & !((done >> t) & 1u) & ((v > best) | ((v == best) & (r < bi)));
      best = take ? v : best;
      bi = take ? r : bi;
    });
    const int mine = bi;
    wave_argmax(best, bi);
    if (lane == 0) {
      s_red[buf][wave].v = best;
      s_red[buf][wave].i = bi;
    }
    if (bi == mine && bi < Rr) {
      // this lane holds the wave's candidate: publish its row (one branch per row slot,
      // each to its own buffer, so the register reads keep constant indices)
      static_for<0, RPT>([&](auto tidx) {
        constexpr int t = decltype(tidx)::value;
        if (bi == tid + t * NT) {
          static_for<0, NB>([&](auto cidx) {
            constexpr int cc = decltype(cidx)::value;
            s_cand[buf][wave][t][cc] = traits<T>::mk(re[t][cc], im[t][cc]);
          });
        }
      });
    }
    __syncthreads();
    RedPair<R> pr[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) pr[k] = s_red[buf][k];
    R bv = pr[0].v;
    int p = pr[0].i;
#pragma unroll
    for (int k = 1; k < NW; ++k) {
      const bool take = (pr[k].v > bv) | ((pr[k].v == bv) & (pr[k].i < p));
      bv = take ? pr[k].v : bv;
      p = take ? pr[k].i : p;
    }
    if (p < 0 || p >= Rr) {
      // a NaN column leaves no candidate: take the first row that is not a pivot yet
      // and publish it through the LDS copy of the panel rows of slot 0 (rare path)
      p = Rr;
      for (int r = 0; r < Rr && p == Rr; ++r) {
        bool used = false;
        for (int q = 0; q < c; ++q) used |= (s_pphys[q] == r);
        if (!used) p = r;
      }
      __syncthreads();
      static_for<0, RPT>([&](auto tidx) {
        constexpr int t = decltype(tidx)::value;
        if (p == tid + t * NT) {
          static_for<0, NB>([&](auto cidx) {
            constexpr int cc = decltype(cidx)::value;
            s_cand[buf][(p % NT) >> 6][t][cc] = traits<T>::mk(re[t][cc], im[t][cc]);
          });
        }
      });
      __syncthreads();
    }
    const T* prow = &s_cand[buf][(p % NT) >> 6][p / NT][0];
    if ((p % NT) == tid) done |= 1u << (p / NT);
    if (tid < NB) s_lu[c][tid] = prow[tid];
    if (tid == 0) s_pphys[c] = p;
    const T pv = prow[c];
    const bool zero = traits<T>::abs2(pv) == 0;
    if (zero && tid == 0) *g.flag = 1;
    const T inv = zero ? traits<T>::zero() : sc_inv(pv);
    // multipliers of the own rows (a pivot row's registers are not read again)
    T l[RPT];
    static_for<0, RPT>([&](auto tidx) {
      constexpr int t = decltype(tidx)::value;
      l[t] = sc_mul(traits<T>::mk(cr[t], ci[t]), inv);
    });
    // chunks of columns: the chunk of the pivot row is read from LDS in one batch
    constexpr int CH = sizeof(T) == 16 ? 4 : 8;
    static_for<0, NB / CH>([&](auto chi) {
      constexpr int cb = decltype(chi)::value * CH;
      if (cb + CH - 1 >= c) {
        R pre[CH], pim[CH];
        static_for<0, CH>([&](auto ui) {
          constexpr int u = decltype(ui)::value;
          const T v = prow[cb + u];
          pre[u] = traits<T>::re(v);
          pim[u] = traits<T>::im(v);
        });
        static_for<0, CH>([&](auto ui) {
          constexpr int u = decltype(ui)::value;
          constexpr int cc = cb + u;
          if (cc == c) {
            static_for<0, RPT>([&](auto tidx) {
              constexpr int t = decltype(tidx)::value;
              re[t][cc] = traits<T>::re(l[t]);
              im[t][cc] = traits<T>::im(l[t]);
            });
          } else if (cc > c) {
            const T pw = traits<T>::mk(pre[u], pim[u]);
            static_for<0, RPT>([&](auto tidx) {
              constexpr int t = decltype(tidx)::value;
              const T nv = sc_fms(traits<T>::mk(re[t][cc], im[t][cc]), l[t], pw);
              re[t][cc] = traits<T>::re(nv);
              im[t][cc] = traits<T>::im(nv);
              if (cc == c + 1) {
                cr[t] = re[t][cc];
                ci[t] = im[t][cc];
              }
            });
          }
        });
      }
    });
  }
  __syncthreads();
  if (wave == 0) panel_moves(g.mv, s_pphys, w);
  pivot_block_inverse<T, NB, NB + 1>(&s_lu[0][0], w, g.pinv);
}

// a - b c with four fused multiply-adds for complex operands
__device__ __forceinline__ float fms4(float a, float b, float c) { return fmaf(-b, c, a); }
__device__ __forceinline__ double fms4(double a, double b, double c) { return fma(-b, c, a); }
__device__ __forceinline__ cf fms4(cf a, cf b, cf c) {
  return {fmaf(-b.x, c.x, fmaf(b.y, c.y, a.x)), fmaf(-b.x, c.y, fmaf(-b.y, c.x, a.y))};
}
__device__ __forceinline__ cd fms4(cd a, cd b, cd c) {
  return {fma(-b.x, c.x, fma(b.y, c.y, a.x)), fma(-b.x, c.y, fma(-b.y, c.x, a.y))};
}
// 1 / a for a pivot: hardware reciprocal (about 1 ulp) in single precision,
// a correctly rounded division in double precision
__device__ __forceinline__ float pivot_inv(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ double pivot_inv(double a) { return 1.0 / a; }
__device__ __forceinline__ cf pivot_inv(cf a) {
  const float r = __builtin_amdgcn_rcpf(a.x * a.x + a.y * a.y);
  return {a.x * r, -a.y * r};
}
__device__ __forceinline__ cd pivot_inv(cd a) {
  const double r = 1.0 / (a.x * a.x + a.y * a.y);
  return {a.x * r, -a.y * r};
}

// Wave-wide (value, row) maximum for pivot search: the largest value, then the
// lowest row index among the lanes holding it; uniform result. Four in-row DPP steps
// and three cross-row steps through readlane for each of the two reductions.
template <class R> __device__ __forceinline__ void wave_pivot_max(R& v, int& i) {
  R m = v;
  m = fmax(m, dpp_v<0xB1>(m));
  m = fmax(m, dpp_v<0x4E>(m));
  m = fmax(m, dpp_v<0x141>(m));
  m = fmax(m, dpp_v<0x140>(m));
  m = fmax(fmax(rdlane(m, 0), rdlane(m, 16)), fmax(rdlane(m, 32), rdlane(m, 48)));
  int k = v == m ? i : 0x7fffffff;
  k = min(k, dpp_i<0xB1>(k));
  k = min(k, dpp_i<0x4E>(k));
  k = min(k, dpp_i<0x141>(k));
  k = min(k, dpp_i<0x140>(k));
  k = min(min(rdlane(k, 0), rdlane(k, 16)), min(rdlane(k, 32), rdlane(k, 48)));
  v = m;
  i = k;
}

// Single-precision pivot search with one reduction: the key of a candidate holds the
// modulus (a non-negative float; -0.5 for NaN, -1 for no candidate) in the high word
// as an order-preserving unsigned integer and the complement of the row in the low
// word, so the largest key is the largest modulus with the lowest row.
__device__ __forceinline__ uint64_t pivot_key(float v, int row) {
  const uint32_t u = __float_as_uint(v);
  const uint32_t hi = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((uint64_t)hi << 32) | (uint64_t)(~(uint32_t)row);
}
__device__ __forceinline__ int key_row(uint64_t k) { return (int)(~(uint32_t)k); }
template <int CTRL> __device__ __forceinline__ uint64_t dpp_u64(uint64_t k) {
  const uint32_t lo = (uint32_t)dpp_i<CTRL>((int)(uint32_t)k);
  const uint32_t hi = (uint32_t)dpp_i<CTRL>((int)(uint32_t)(k >> 32));
  return ((uint64_t)hi << 32) | lo;
}
// wave-wide maximum of the keys, uniform: four in-row DPP steps, then the four rows
__device__ __forceinline__ uint64_t wave_max_key(uint64_t k) {
  uint64_t o;
  o = dpp_u64<0xB1>(k);
  k = o > k ? o : k;
  o = dpp_u64<0x4E>(k);
  k = o > k ? o : k;
  o = dpp_u64<0x141>(k);
  k = o > k ? o : k;
  o = dpp_u64<0x140>(k);
  k = o > k ? o : k;
  uint64_t r[4];
  static_for<0, 4>([&](auto qq) {
    constexpr int q = decltype(qq)::value;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)k, 16 * q);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(k >> 32), 16 * q);
    r[q] = ((uint64_t)hi << 32) | lo;
  });
  const uint64_t a = r[0] > r[1] ? r[0] : r[1], b = r[2] > r[3] ? r[2] : r[3];
  return a > b ? a : b;
}

// Pinv = A11^{-1} for the pivot block of a panel, A11(c, :) = the original panel
// row of the pivot of column c (rows in pivot order), by Gauss-Jordan elimination
// without further interchanges: its pivots are those of the panel's LU. Every
// thread keeps EPT elements of the w x w block in registers; per step one barrier
// (the pivot row and column go through double-buffered LDS).
template <class T, int NB, int NT>
__device__ __forceinline__ void pivot_block_gj(const GjDesc<T>& g, int j0, int base, int w, const int* pphys,
                                               T (*s_row)[NB], T (*s_col)[NB]) {
  constexpr int EPT = (NB * NB + NT - 1) / NT;
  const int tid = threadIdx.x;
  T a[EPT];
  int ei[EPT], ej[EPT];
  static_for<0, EPT>([&](auto qq) {
    constexpr int q = decltype(qq)::value;
    const int e = tid + q * NT;
    ei[q] = e % NB;
    ej[q] = e / NB;
    const bool in = ei[q] < w && ej[q] < w;
    a[q] = in ? g.M[(base + pphys[in ? ei[q] : 0]) + (size_t)(j0 + (in ? ej[q] : 0)) * g.rows] : traits<T>::zero();
  });
  for (int k = 0; k < w; ++k) {
    const int b = k & 1;
    static_for<0, EPT>([&](auto qq) {
      constexpr int q = decltype(qq)::value;
      if (ei[q] == k && ej[q] < w) s_row[b][ej[q]] = a[q];
      if (ej[q] == k && ei[q] < w) s_col[b][ei[q]] = a[q];
    });
    __syncthreads();
    const T p = s_row[b][k];
    const bool zp = traits<T>::abs2(p) == 0;
    if (zp && tid == 0) *g.flag = 1;
    const T ip = zp ? traits<T>::zero() : pivot_inv(p);
    static_for<0, EPT>([&](auto qq) {
      constexpr int q = decltype(qq)::value;
      const int i = ei[q], j = ej[q];
      if (i < w && j < w) {
        const T rk = sc_mul(s_row[b][j], ip);  // scaled pivot row entry
        const T cik = s_col[b][i];
        T v;
        if (i == k) v = j == k ? ip : rk;
        else v = j == k ? -sc_mul(cik, ip) : fms4(a[q], cik, rk);
        a[q] = v;
      }
    });
  }
  static_for<0, EPT>([&](auto qq) {
    constexpr int q = decltype(qq)::value;
    if (ei[q] < w && ej[q] < w) g.pinv[ei[q] + ej[q] * w] = a[q];
  });
}

// Register-resident panel LU with a compact column loop: NT threads, thread tid
// owns rows tid + t * NT (t < RPT) and keeps, in slots 0 .. NB - 1, the values of
// columns c .. c + NB - 1 of its rows (column c of the loop in slot 0). The update of
// column c shifts every row left by one slot in the same fused multiply-adds, so
// every register index is a compile-time constant and the loop body has no branch
// on c. Only the pivots are needed from the panel; Pinv is recomputed from the
// original pivot rows at the end (pivot_block_gj). Per column: each wave's best
// candidate (largest modulus, lowest row on ties; a NaN modulus ranks below every
// number) and its row go to LDS, one barrier, then every thread reduces the wave
// partials and updates its rows with the pivot row. The search and the
// elimination run in the matrix's own precision, so the pivots are those of
// partial pivoting in that precision.
// The pivot search of the compact panel: the Rr candidate rows rowof(0 .. Rr - 1)
// of M (Rr <= RPT * NT), columns j0 .. j0 + w - 1; s_pphys[c] receives the index
// r of the pivot of column c. Every thread of the block takes part. An exactly zero
// pivot sets *zflag (when given): the panel is singular if the search covers all
// its candidate rows, not when it covers one chunk of them.
template <class T, int NB, int RPT, int NT, class RowOf>
__device__ __forceinline__ void rot_search(const GjDesc<T>& g, int j0, int w, int Rr, RowOf rowof, int* s_pphys,
                                           int* zflag) {
  using S = T;
  using R = typename traits<S>::real;
  constexpr bool CPLX = traits<T>::cplx;
  constexpr int NW = NT / 64;
  __shared__ RedPair<R> s_red[2][NW];
  __shared__ uint64_t s_key[2][NW];
  constexpr bool KEYS = std::is_same<R, float>::value;  // one 64-bit reduction
  __shared__ R s_cre[2][NW][NB];
  __shared__ R s_cim[2][NW][CPLX ? NB : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  R re[RPT][NB], im[RPT][NB];
  static_for<0, RPT>([&](auto tidx) {
    constexpr int t = decltype(tidx)::value;
    const int r = tid + t * NT;
    const int rr = rowof(min(r, Rr - 1));
    static_for<0, NB>([&](auto ci) {
      constexpr int cc = decltype(ci)::value;
      const T v = g.M[rr + (size_t)(j0 + min(cc, w - 1)) * g.rows];
      const bool keep = r < Rr && cc < w;
      re[t][cc] = keep ? R(traits<T>::re(v)) : R(0);
      im[t][cc] = keep ? R(traits<T>::im(v)) : R(0);
    });
  });
  unsigned done = 0;  // bit t: own row t is a pivot row
  for (int c = 0; c < w; ++c) {
    const int buf = c & 1;
    R best = -1;
    int bi = 0x7fffffff;
    static_for<0, RPT>([&](auto tidx) {
      constexpr int t = decltype(tidx)::value;
      const int r = tid + t * NT;
      R v = re[t][0] * re[t][0] + im[t][0] * im[t][0];
      v = v == v ? v : R(-0.5);
      // rows grow with t, so a strict comparison keeps the lowest row on ties
      const bool take = (r < Rr) & !((done >> t) & 1u) & (v > best);
      best = take ? v : best;
      bi = take ? r : bi;
    });
    const int mine = bi;
    if constexpr (KEYS) {
      const uint64_t key = wave_max_key(pivot_key(best, bi));
      bi = key_row(key);
      if (lane == 0) s_key[buf][wave] = key;
    } else {
      wave_pivot_max(best, bi);
      if (lane == 0) {
        s_red[buf][wave].v = best;
        s_red[buf][wave].i = bi;
      }
    }
    if (bi == mine && bi < Rr) {
      // this lane holds the wave's candidate: publish its row (one branch per row
      // slot, so that the register reads keep constant indices)
      static_for<0, RPT>([&](auto tidx) {
        constexpr int t = decltype(tidx)::value;
        if (bi == tid + t * NT) {
          static_for<0, NB>([&](auto ci) {
            constexpr int cc = decltype(ci)::value;
            s_cre[buf][wave][cc] = re[t][cc];
            if constexpr (CPLX) s_cim[buf][wave][cc] = im[t][cc];
          });
        }
      });
    }
    __syncthreads();
    int p;
    if constexpr (KEYS) {
      uint64_t kmax = s_key[buf][0];
      static_for<1, NW>([&](auto kk) {
        const uint64_t o = s_key[buf][decltype(kk)::value];
        kmax = o > kmax ? o : kmax;
      });
      p = key_row(kmax);
    } else {
      RedPair<R> pr[NW];
      static_for<0, NW>([&](auto kk) { pr[decltype(kk)::value] = s_red[buf][decltype(kk)::value]; });
      R bv = pr[0].v;
      p = pr[0].i;
      static_for<1, NW>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        const bool take = (pr[k].v > bv) | ((pr[k].v == bv) & (pr[k].i < p));
        bv = take ? pr[k].v : bv;
        p = take ? pr[k].i : p;
      });
    }
    const int pwv = (p % NT) >> 6;
    const R* pre = &s_cre[buf][pwv][0];
    const R* pim = &s_cim[buf][CPLX ? pwv : 0][0];
    if ((p % NT) == tid) done |= 1u << (p / NT);
    if (tid == 0) s_pphys[c] = p;
    // the whole pivot row into registers at once: one LDS round trip per column
    R prr[NB], pri[NB];
    static_for<0, NB>([&](auto ci) {
      constexpr int k = decltype(ci)::value;
      prr[k] = pre[k];
      pri[k] = CPLX ? pim[k] : R(0);
    });
    __builtin_amdgcn_sched_barrier(0);
    const S pv = traits<S>::mk(prr[0], pri[0]);
    const bool zero = traits<S>::abs2(pv) == 0;
    if (zero && tid == 0 && zflag) *zflag = 1;
    const S inv = zero ? traits<S>::zero() : pivot_inv(pv);
    S l[RPT];
    static_for<0, RPT>([&](auto tidx) {
      constexpr int t = decltype(tidx)::value;
      l[t] = sc_mul(traits<S>::mk(re[t][0], im[t][0]), inv);
    });
    // update and shift: slot k takes column c + 1 + k
    static_for<0, NB - 1>([&](auto ci) {
      constexpr int k = decltype(ci)::value;
      const S pw = traits<S>::mk(prr[k + 1], pri[k + 1]);
      static_for<0, RPT>([&](auto tidx) {
        constexpr int t = decltype(tidx)::value;
        const S nv = fms4(traits<S>::mk(re[t][k + 1], im[t][k + 1]), l[t], pw);
        re[t][k] = traits<S>::re(nv);
        im[t][k] = traits<S>::im(nv);
      });
    });
    static_for<0, RPT>([&](auto tidx) {
      constexpr int t = decltype(tidx)::value;
      re[t][NB - 1] = R(0);
      im[t][NB - 1] = R(0);
    });
  }
}

// the end of a panel step once its pivots (relative to base) are in s_pphys: the
// row permutation (gj_rows_kernel is told to leave it), the net row movement and
// Pinv from the original pivot rows
template <class T, int NB, int NT>
__device__ __forceinline__ void panel_finish(const GjDesc<T>& g, int j0, int base, int w, int* s_pphys) {
  __shared__ T s_row[2][NB], s_col[2][NB];
  const int tid = threadIdx.x;
  if (g.rowperm && j0 == 0)
    for (int i = tid; i < g.rows; i += NT) g.rowperm[i] = i;
  __syncthreads();
  if ((tid >> 6) == 0) panel_moves(g.mv, s_pphys, w, g.rowperm, base);
  pivot_block_gj<T, NB, NT>(g, j0, base, w, s_pphys, s_row, s_col);
}

template <class T, int NB, int RPT, int NT>
__global__ __launch_bounds__(NT) void gj_panel_rot_kernel(const GjDesc<T>* __restrict__ descs, int j0, int nb) {
  const GjDesc<T> g = descs[blockIdx.x];
  if (j0 >= g.n) return;
  const int w = min(nb, g.n - j0);
  const int base = g.poff + j0;  // first candidate row
  const int Rr = g.rows - base;  // candidate rows, >= w
  __shared__ int s_pphys[NB];
  rot_search<T, NB, RPT, NT>(g, j0, w, Rr, [&](int r) { return base + r; }, s_pphys, g.flag);
  panel_finish<T, NB, NT>(g, j0, base, w, s_pphys);
}

// Tournament pivoting for panels taller than one compact kernel holds (the
// communication-avoiding LU of Grigori, Demmel and Xiang): the candidate rows are
// cut into chunks of RPT * NT rows, each chunk picks w local pivots by partial
// pivoting on its own rows (gj_tourn_local_kernel, one workgroup per chunk and
// box), and partial pivoting on the original values of the stacked local pivots
// picks the panel's pivots (gj_tourn_final_kernel, one workgroup per box).
// cand[(box * nch + chunk) * NB + c]: local pivot c of the chunk, relative to the
// panel's first candidate row, or -1.
template <class T, int NB, int RPT, int NT>
__global__ __launch_bounds__(NT) void gj_tourn_local_kernel(const GjDesc<T>* __restrict__ descs, int j0, int nb,
                                                            int nch, int* __restrict__ cand) {
  const GjDesc<T> g = descs[blockIdx.y];
  int* out = cand + ((size_t)blockIdx.y * nch + blockIdx.x) * NB;
  const int w = j0 < g.n ? min(nb, g.n - j0) : 0;
  const int base = g.poff + j0;
  const int r0 = (int)blockIdx.x * RPT * NT;
  const int cnt = w > 0 ? min(RPT * NT, g.rows - base - r0) : 0;
  if (cnt <= 0) {
    if (threadIdx.x < NB) out[threadIdx.x] = -1;
    return;
  }
  __shared__ int s_pphys[NB];
  const int wl = min(w, cnt);
  rot_search<T, NB, RPT, NT>(g, j0, wl, cnt, [&](int r) { return base + r0 + r; }, s_pphys, nullptr);
  __syncthreads();
  if (threadIdx.x < NB) out[threadIdx.x] = threadIdx.x < wl ? r0 + s_pphys[threadIdx.x] : -1;
}

template <class T, int NB, int RPT, int NT>
__global__ __launch_bounds__(NT) void gj_tourn_final_kernel(const GjDesc<T>* __restrict__ descs, int j0, int nb,
                                                            int nch, const int* __restrict__ cand) {
  const GjDesc<T> g = descs[blockIdx.x];
  if (j0 >= g.n) return;
  const int w = min(nb, g.n - j0);
  const int base = g.poff + j0;
  __shared__ int s_cl[RPT * NT];  // the valid candidates, relative to base
  __shared__ int s_wn[NT / 64];
  __shared__ int s_pphys[NB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // stable compaction of the valid candidates (chunk order, then local pivot
  // order), NT entries per round: the position of an entry is the number of valid
  // entries before it (ballots within a wave, wave counts through LDS)
  const int nc = nch * NB;
  const int* cb = cand + (size_t)blockIdx.x * nc;
  int m = 0;
  for (int c0 = 0; c0 < nc; c0 += NT) {
    const int i = c0 + tid;
    const int v = i < nc ? cb[i] : -1;
    const bool ok = v >= 0;
    const unsigned long long mask = __ballot(ok);
    if (lane == 0) s_wn[wave] = __popcll(mask);
    __syncthreads();
    int before = m + __popcll(mask & ((1ull << lane) - 1));
    int total = 0;
    static_for<0, NT / 64>([&](auto ww) {
      constexpr int q = decltype(ww)::value;
      const int c = s_wn[q];
      if (q < wave) before += c;
      total += c;
    });
    if (ok && before < RPT * NT) s_cl[before] = v;
    m += total;
    __syncthreads();
  }
  m = min(m, RPT * NT);
  rot_search<T, NB, RPT, NT>(g, j0, w, m, [&](int r) { return base + s_cl[r]; }, s_pphys, g.flag);
  __syncthreads();
  const int p = tid < w ? s_cl[s_pphys[tid]] : 0;
  __syncthreads();
  if (tid < w) s_pphys[tid] = p;
  panel_finish<T, NB, NT>(g, j0, base, w, s_pphys);
}


// Row interchanges, pivot-row scaling and the saved panel columns; grid
// (ntx column tiles of 64 + row blocks of 256, box). The panel columns of M are
// not touched here: the trailing GEMM rewrites them completely (beta = 0 on the
// panel's column window), so the row blocks can copy them to csave concurrently.
//   column tile: interchanges on its columns outside the panel, then
//                R' = Pinv * (pivot rows) into rbuf (Pinv itself for panel columns)
//                and zeros into the pivot rows of M;
//   row block:   csave = panel columns of the interchanged M, pivot block -I.
// With C = M - csave R' (beta 0 on the panel window) this gives the pivot rows R',
// the other rows M - csave R', and the panel columns -csave Pinv / Pinv.
template <class T>
__global__ __launch_bounds__(256) void gj_rows_kernel(const GjDesc<T>* __restrict__ descs,
                                                      int j0, int nb, int ntx, int rp_done) {
  using R = typename traits<T>::real;
  const GjDesc<T> g = descs[blockIdx.y];
  if (j0 >= g.n) return;
  const int w = min(nb, g.n - j0);
  const int base = g.poff + j0;  // pivot row of panel column 0
  const int tid = threadIdx.x;
  __shared__ int s_mv[2 * 64];
  const int nm = g.mv[0];
  if (tid < 2 * nm) s_mv[tid] = g.mv[1 + tid];
  if ((int)blockIdx.x >= ntx) {
    // ---- row block: csave rows [r0, r0 + 256)
    const int r0 = ((int)blockIdx.x - ntx) * 256;
    if (r0 >= g.rows) return;
    __shared__ int s_src[256];
    s_src[tid] = -1;
    __syncthreads();
    if (tid < nm) {
      const int dst = base + s_mv[2 * tid];
      if (dst >= r0 && dst < r0 + 256) s_src[dst - r0] = base + s_mv[2 * tid + 1];
    }
    __syncthreads();
    const int r = r0 + tid;
    if (r >= g.rows) return;
    const bool pivrow = r >= base && r < base + w;
    const int src = s_src[tid] >= 0 ? s_src[tid] : r;
    constexpr int U = 8;
    for (int cb = 0; cb < w; cb += U) {
      R vr[U], vi[U];
      static_for<0, U>([&](auto uu) {
        constexpr int u = decltype(uu)::value;
        const T x = (cb + u < w && !pivrow) ? g.M[src + (size_t)(j0 + cb + u) * g.rows] : traits<T>::zero();
        vr[u] = traits<T>::re(x);
        vi[u] = traits<T>::im(x);
      });
      static_for<0, U>([&](auto uu) {
        constexpr int u = decltype(uu)::value;
        if (cb + u < w) {
          const T x = pivrow ? (r - base == cb + u ? traits<T>::mk(-1.0, 0.0) : traits<T>::zero())
                             : traits<T>::mk(vr[u], vi[u]);
          g.csave[r + (size_t)(cb + u) * g.rows] = x;
        }
      });
    }
    return;
  }
  // ---- column tile
  const int c0 = blockIdx.x * 64;
  if (c0 >= g.W) return;
  const int cw = min(64, g.W - c0);
  __shared__ T s_pinv[32 * 32];
  __shared__ T s_seg[32][65];
  static_for<0, 4>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    const int i = tid + k * 256;
    if (i < w * w) s_pinv[i] = g.pinv[i];
  });
  __syncthreads();
  // 1. loads, all from M as it is before the step: the rows that the moves carry
  //    below the pivot block (dst >= w; every other move ends in a pivot position,
  //    whose row is replaced by R'), and the pivot rows' segment from wherever the
  //    pivot rows sit now
  constexpr int PER = 64 * 64 / 256;  // up to 2 nb = 64 moves of 64 columns
  R vr[PER], vi[PER];
  const int tot = nm * cw;
  static_for<0, PER>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    const int idx = tid + k * 256;
    const int e = nm > 0 ? idx % nm : 0;
    const int col = c0 + (nm > 0 ? idx / nm : 0);
    const bool act = idx < tot && s_mv[2 * e] >= w && (col < j0 || col >= j0 + w);
    const T x = act ? g.M[(base + s_mv[2 * e + 1]) + (size_t)col * g.rows] : traits<T>::zero();
    vr[k] = traits<T>::re(x);
    vi[k] = traits<T>::im(x);
  });
  for (int idx = tid; idx < w * cw; idx += 256) {
    const int i = idx % w, c = idx / w;
    int src = i;  // the pivot of column i sits at base + src before the moves
    for (int e = 0; e < nm; ++e)
      if (s_mv[2 * e] == i) src = s_mv[2 * e + 1];
    s_seg[i][c] = g.M[(base + src) + (size_t)(c0 + c) * g.rows];
  }
  if (!rp_done && g.rowperm && blockIdx.x == 0) {
    if (j0 == 0)
      for (int i = tid; i < g.rows; i += 256) g.rowperm[i] = i;
    __syncthreads();
    const int rp = tid < nm ? g.rowperm[base + s_mv[2 * tid + 1]] : 0;
    __syncthreads();
    if (tid < nm) g.rowperm[base + s_mv[2 * tid]] = rp;
  }
  __syncthreads();
  // 2. stores: the carried rows, R' = Pinv * segment into rbuf, zeros in the pivot rows
  static_for<0, PER>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    const int idx = tid + k * 256;
    const int e = nm > 0 ? idx % nm : 0;
    const int col = c0 + (nm > 0 ? idx / nm : 0);
    if (idx < tot && s_mv[2 * e] >= w && (col < j0 || col >= j0 + w))
      g.M[(base + s_mv[2 * e]) + (size_t)col * g.rows] = traits<T>::mk(vr[k], vi[k]);
  });
  for (int idx = tid; idx < w * cw; idx += 256) {
    const int i = idx % w, c = idx / w;
    const int gc = c0 + c;
    T v;
    if (gc >= j0 && gc < j0 + w) {
      v = s_pinv[i + (gc - j0) * w];
    } else {
      v = traits<T>::zero();
      for (int k = 0; k < w; ++k) v = v + sc_mul(s_pinv[i + k * w], s_seg[k][c]);
      g.M[(base + i) + (size_t)gc * g.rows] = traits<T>::zero();
    }
    g.rbuf[i + (size_t)gc * w] = v;
  }
}

// ------------------------------------------------------------- second-level blocking
// For large blocks the pivot columns are taken in blocks of wo (64): the block's
// columns of M (all rows) are copied to pb and eliminated there with the panel
// kernels above (pivot rows from poff = J on); then the block's net row movement
// and one product M += pb * rbuf apply the whole block to the other columns. In
// pb the pivot rows end up holding the inverse of the pivot block and the other
// rows -A21 A11^{-1}, so with the pivot rows of M moved into rbuf (and zeroed in
// M) the product is exactly the block's Gauss-Jordan update; the identity in
// rbuf's block columns (beta = 0 there) writes pb back into M.

constexpr int GJ_BLOCK_MAX = 256;  // widest block (at most 2 GJ_BLOCK_MAX moved rows)
constexpr int GJ_BLOCK_TILE = 16;  // columns per workgroup of gj_block_rows

// pb = M(:, J : J + wb); grid (chunks, box)
template <class T>
__global__ __launch_bounds__(256) void gj_block_copy_kernel(const GjDesc<T>* __restrict__ descs, int J, int wo) {
  const GjDesc<T> g = descs[blockIdx.y];
  if (J >= g.n) return;
  const int wb = min(wo, g.n - J);
  const int64_t tot = (int64_t)g.rows * wb;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256)
    g.pb[e] = g.M[(e % g.rows) + (size_t)(J + e / g.rows) * g.rows];
}

// The block's net row movement from its row permutation rp_in (positions >= J):
// (dst, src) pairs relative to J into mv, and the matrix's row permutation
// updated with them (initialised at J = 0). One workgroup per box; a block of wb
// pivot columns moves at most 2 wb rows.
template <class T>
__global__ __launch_bounds__(256) void gj_block_moves_kernel(const GjDesc<T>* __restrict__ descs, int J) {
  const GjDesc<T> g = descs[blockIdx.x];
  if (J >= g.n) return;
  __shared__ int s_cnt;
  __shared__ int s_dst[2 * GJ_BLOCK_MAX], s_src[2 * GJ_BLOCK_MAX];
  const int tid = threadIdx.x;
  if (tid == 0) s_cnt = 0;
  if (J == 0)
    for (int i = tid; i < g.rows; i += 256) g.rowperm[i] = i;
  __syncthreads();
  for (int i = J + tid; i < g.rows; i += 256) {
    const int src = g.rp_in[i];
    if (src != i) {
      const int k = atomicAdd(&s_cnt, 1);
      if (k < 2 * GJ_BLOCK_MAX) {
        s_dst[k] = i;
        s_src[k] = src;
      }
    }
  }
  __syncthreads();
  const int nm = min(s_cnt, 2 * GJ_BLOCK_MAX);
  constexpr int MPT = 2 * GJ_BLOCK_MAX / 256;  // moves per thread
  int v[MPT];
  static_for<0, MPT>([&](auto uu) {
    constexpr int u = decltype(uu)::value;
    const int i = tid + u * 256;
    v[u] = i < nm ? g.rowperm[s_src[i]] : 0;
  });
  __syncthreads();
  static_for<0, MPT>([&](auto uu) {
    constexpr int u = decltype(uu)::value;
    const int i = tid + u * 256;
    if (i < nm) {
      g.rowperm[s_dst[i]] = v[u];
      g.mv[1 + 2 * i] = s_dst[i] - J;
      g.mv[2 + 2 * i] = s_src[i] - J;
    }
  });
  if (tid == 0) g.mv[0] = nm;
}

// The block's moves on the columns outside [J, J + wb) (all moved entries of the
// tile loaded, then stored), then the pivot rows J .. J + wb - 1 of those columns
// copied to rbuf (wb x W) and zeroed in M; rbuf's block columns get the identity.
// ldu: the block LDU form, whose columns left of the block keep their pivot rows
// (only the moves apply there). Grid (GJ_BLOCK_TILE-column tiles, box).
template <class T>
__global__ __launch_bounds__(256) void gj_block_rows_kernel(const GjDesc<T>* __restrict__ descs, int J, int wo,
                                                            int ldu) {
  using R = typename traits<T>::real;
  const GjDesc<T> g = descs[blockIdx.y];
  if (J >= g.n) return;
  const int wb = min(wo, g.n - J);
  const int c0 = blockIdx.x * GJ_BLOCK_TILE;
  if (c0 >= g.W) return;
  const int cw = min(GJ_BLOCK_TILE, g.W - c0);
  const int tid = threadIdx.x;
  __shared__ int s_mv[4 * GJ_BLOCK_MAX];
  const int nm = min(g.mv[0], 2 * GJ_BLOCK_MAX);
  for (int i = tid; i < 2 * nm; i += 256) s_mv[i] = g.mv[1 + i];
  __syncthreads();
  {
    constexpr int PER = 2 * GJ_BLOCK_MAX * GJ_BLOCK_TILE / 256;
    R vr[PER], vi[PER];
    const int tot = nm * cw;
    static_for<0, PER>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      const int idx = tid + k * 256;
      const int e = nm > 0 ? idx % nm : 0;
      const int col = c0 + (nm > 0 ? idx / nm : 0);
      const bool act = idx < tot && (col < J || col >= J + wb);
      const T x = act ? g.M[(J + s_mv[2 * e + 1]) + (size_t)col * g.rows] : traits<T>::zero();
      vr[k] = traits<T>::re(x);
      vi[k] = traits<T>::im(x);
    });
    __syncthreads();
    static_for<0, PER>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      const int idx = tid + k * 256;
      const int e = nm > 0 ? idx % nm : 0;
      const int col = c0 + (nm > 0 ? idx / nm : 0);
      if (idx < tot && (col < J || col >= J + wb))
        g.M[(J + s_mv[2 * e]) + (size_t)col * g.rows] = traits<T>::mk(vr[k], vi[k]);
    });
  }
  __syncthreads();
  for (int idx = tid; idx < wb * cw; idx += 256) {
    const int i = idx % wb, col = c0 + idx / wb;
    if (ldu && col < J) continue;
    T* mp = g.M + (J + i) + (size_t)col * g.rows;
    if (col >= J && col < J + wb) {
      g.rbuf[i + (size_t)col * wb] = col - J == i ? traits<T>::one() : traits<T>::zero();
    } else {
      g.rbuf[i + (size_t)col * wb] = *mp;
      *mp = traits<T>::zero();
    }
  }
}

// Explicit inverse from the pivoted one: A^{-1} = (P A)^{-1} P, i.e. column
// rowperm[i] of A^{-1} is column i of M; written to out (n x n, ld n). Grid
// (column tiles, box); one thread per row of a 64-column tile.
template <class T>
__global__ __launch_bounds__(256) void gj_colperm_kernel(const GjDesc<T>* __restrict__ descs, T* const* outs) {
  const GjDesc<T> g = descs[blockIdx.y];
  T* out = outs[blockIdx.y];
  const int c0 = blockIdx.x * 64;
  if (c0 >= g.n) return;
  for (int r = threadIdx.x; r < g.n; r += 256)
    for (int i = c0; i < min(c0 + 64, g.n); ++i) out[r + (size_t)g.rowperm[i] * g.n] = g.M[r + (size_t)i * g.n];
}

}  // namespace hss
