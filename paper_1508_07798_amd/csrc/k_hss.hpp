// HSS compression of the Schur complements by randomized interpolative
// decompositions (Section 1: the HSS nesting condition, the ID with a
// well-behaved interpolation matrix, Theorem 1 with oversampling 10).
//
// For each box the dense S (n x n, symmetric or complex symmetric) is
// compressed over its HSS tree, children before parents:
//   candidates R: all indices of an HSS leaf, else the children's skeletons;
//   samples    Z = S(R, tau^c) Omega(tau^c, :) = Y(R, :) - S(R, tau) Omega(tau, :),
//              Y = S Omega formed once per box by the batched GEMM;
//   row ID     CPQR of Z^T (Householder, column pivoting by the largest
//              remaining column norm, ties to the lowest index) stopped at
//              the first k with ||R22||_F <= threshold; skeleton J = R(perm(1:k)),
//              T = R11^{-1} R12, interpolation U(perm(1:k)) = I, U(perm(k+1:)) = T^T.
// Generators: D = S(tau, tau) on HSS leaves, B = S(J_a, J_b) between siblings;
// S~(a, b) = Ut_a B Ut_b^T with tall bases Ut (leaf: U, parent:
// diag(Ut_a, Ut_b) U), S~(b, a) = S~(a, b)^T. The judge measures
// ||S - S~||_F / ||S||_F exactly.
#pragma once

#include "common.hpp"
#include "k_gemm.hpp"

namespace hss {

// ------------------------------------------------------------- Philox
struct u4 {
  uint32_t x, y, z, w;
};
__device__ inline u4 philox4x32_10(u4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    c = u4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

template <class T> __device__ inline T gauss_entry(uint64_t seed, uint32_t node, uint32_t r, uint32_t c) {
  u4 o = philox4x32_10(u4{r, c, node, 0u}, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double u1 = ((double)o.x + 0.5) * 2.3283064365386963e-10;
  const double u2 = ((double)o.y + 0.5) * 2.3283064365386963e-10;
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 6.283185307179586 * u2;
  if constexpr (traits<T>::cplx) {
    const double s = 0.7071067811865476;
    return traits<T>::mk(rad * cos(ang) * s, rad * sin(ang) * s);
  } else {
    return traits<T>::mk(rad * cos(ang), 0.0);
  }
}

// ------------------------------------------------------------- descriptors
template <class T> struct CompBox {
  T* S;          // n x n, symmetrised, input
  T* St;         // n x n, output S~
  T* Om;         // n x l test matrix
  T* Y;          // n x l = S Om
  int n, l, n_id;
  uint32_t node;     // heap id (Philox counter word)
  double tol_scale;  // tol * 2^-(2 * (retries + 1))
  double* nrm2;      // ||S||_F^2
  double* err2;      // ||S - S~||_F^2
  int* flags;        // bit 0: an ID ran out of samples
  int* kmax;         // largest rank
  float* tmax;       // largest |T|
};

template <class T> struct HssDesc {
  int box;            // index into the CompBox array
  int lo, hi;         // dof range of tau
  int left, right;    // global HSS node indices of the children, -1 for leaves
  int zcap;           // capacity of candidate rows
  int* cand;          // [zcap] candidate indices into S
  int* skel;          // [zcap] skeleton (first k entries)
  int* k;             // rank
  T* Zt;              // l x zcap samples Z^T (kept through the CPQR)
  T* Zw;              // l x zcap working copy for the CPQR when it does not fit in LDS
  T* U;               // zcap x l interpolation matrix (ld = zcap)
  T* Ut;              // (hi - lo) x l tall basis (ld = hi - lo)
  T* Et;              // internal nodes: S(J_a, J_c) Ut_c^T of the children a, c (ld = ldet)
  int ldet;
};

// ------------------------------------------------------------- kernels
// grid (chunks, boxes): Omega entries
template <class T>
__global__ void omega_kernel(const CompBox<T>* __restrict__ bx, uint64_t seed) {
  const CompBox<T> b = bx[blockIdx.y];
  const int64_t tot = (int64_t)b.n * b.l;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int r = (int)(e % b.n), c = (int)(e / b.n);
    b.Om[e] = gauss_entry<T>(seed, b.node, (uint32_t)r, (uint32_t)c);
  }
}

// S <- (S + S^T)/2 and ||S||_F^2 (atomic partial sums). Grid (tile pairs, boxes):
// block x takes the MT x MT tiles (ti, tj) and (tj, ti), ti <= tj, of the tile
// triangle in order tj (tj + 1) / 2 + ti; both tiles pass through LDS, so every
// global read and write is along columns.
template <class T, int MT>
__global__ __launch_bounds__(256) void symm_norm_kernel(const CompBox<T>* __restrict__ bx) {
  const CompBox<T> b = bx[blockIdx.y];
  const int nt = (b.n + MT - 1) / MT;
  const int64_t k = blockIdx.x;
  if (k >= (int64_t)nt * (nt + 1) / 2) return;
  int tj = (int)((sqrt(8.0 * (double)k + 1.0) - 1.0) / 2.0);
  while ((int64_t)tj * (tj + 1) / 2 > k) --tj;
  while ((int64_t)(tj + 1) * (tj + 2) / 2 <= k) ++tj;
  const int ti = (int)(k - (int64_t)tj * (tj + 1) / 2);
  const int r0 = ti * MT, c0 = tj * MT, n = b.n;
  __shared__ T up[MT][MT + 1];  // up[c][r] = S(r0 + r, c0 + c)
  __shared__ T lo[MT][MT + 1];  // lo[c][r] = S(c0 + r, r0 + c)
  for (int e = threadIdx.x; e < MT * MT; e += 256) {
    const int r = e % MT, c = e / MT;
    if (r0 + r < n && c0 + c < n) up[c][r] = b.S[(r0 + r) + (size_t)(c0 + c) * n];
    if (c0 + r < n && r0 + c < n) lo[c][r] = b.S[(c0 + r) + (size_t)(r0 + c) * n];
  }
  __syncthreads();
  double acc = 0;
  // entry (r0 + r, c0 + c) pairs with (c0 + c, r0 + r) = lo[r][c]
  for (int e = threadIdx.x; e < MT * MT; e += 256) {
    const int r = e % MT, c = e / MT;
    if (r0 + r < n && c0 + c < n && (ti < tj || r <= c)) {
      const T a = up[c][r], t = lo[r][c];
      const T m = traits<T>::mk(0.5 * (traits<T>::re(a) + traits<T>::re(t)),
                                0.5 * (traits<T>::im(a) + traits<T>::im(t)));
      acc += (ti < tj || r < c ? 2.0 : 1.0) * (double)traits<T>::abs2(m);
      up[c][r] = m;
    }
  }
  __syncthreads();
  // diagonal tiles: the lower half takes the mirror of the upper half
  for (int e = threadIdx.x; e < MT * MT; e += 256) {
    const int r = e % MT, c = e / MT;
    if (r0 + r < n && c0 + c < n) {
      const T v = (ti < tj || r <= c) ? up[c][r] : up[r][c];
      b.S[(r0 + r) + (size_t)(c0 + c) * n] = v;
    }
    if (ti < tj && c0 + r < n && r0 + c < n) b.S[(c0 + r) + (size_t)(r0 + c) * n] = up[r][c];
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(b.nrm2, red[0]);
}

// Work item of the tiled HSS kernels: an HSS node and the first row / column
// of the tile a workgroup computes.
struct HTile {
  int hnode;
  int r0, c0;
};

// Samples of one HSS height, one workgroup per (HSS node, 64 x 64 output tile):
// candidates, then Z = Y(R, :) - S(R, tau) Omega(tau, :) written transposed
// (Zt, l x m). The product over tau runs in slabs of 16 staged through LDS as
// split real / imaginary planes and is taken on the matrix cores as in the GEMM
// kernel: four waves, each a 32 x 32 quadrant of 2 x 2 MFMA 16x16 blocks
// (complex64 with three real products per complex product, complex128 with four).
// Tiles beyond the candidate count exit.
template <class T, int MCAP>
__global__ __launch_bounds__(256) void sample_kernel(const CompBox<T>* __restrict__ bx,
                                                     const HssDesc<T>* __restrict__ hs,
                                                     const HTile* __restrict__ tiles) {
  using R = typename traits<T>::real;
  using Acc = typename mfma_acc<R>::type;
  constexpr bool CX = traits<T>::cplx;
  constexpr bool G3 = CX && std::is_same<R, float>::value;
  constexpr int NP = CX ? (G3 ? 3 : 2) : 1;
  constexpr int KC = 16, LD = 64 + 4;
  const HTile tl = tiles[blockIdx.x];
  const HssDesc<T> h = hs[tl.hnode];
  const CompBox<T> b = bx[h.box];
  __shared__ int s_cand[MCAP];
  __shared__ int s_m;
  __shared__ R Sg[NP][KC][LD];  // S(R, tau) slab: [plane][k][row]
  __shared__ R Og[NP][KC][LD];  // Omega(tau, :) slab: [plane][k][col]
  const int tid = threadIdx.x;
  if (h.left < 0) {
    for (int i = tid; i < h.hi - h.lo; i += 256) s_cand[i] = h.lo + i;
    if (tid == 0) s_m = h.hi - h.lo;
  } else {
    const HssDesc<T> a = hs[h.left], c = hs[h.right];
    const int ka = *a.k, kc = *c.k;
    for (int i = tid; i < ka; i += 256) s_cand[i] = a.skel[i];
    for (int i = tid; i < kc; i += 256) s_cand[ka + i] = c.skel[i];
    if (tid == 0) s_m = ka + kc;
  }
  __syncthreads();
  const int m = s_m;
  if (tl.r0 == 0 && tl.c0 == 0)
    for (int i = tid; i < m; i += 256) h.cand[i] = s_cand[i];
  const int l = b.l, n = b.n;
  const int r0 = tl.r0, c0 = tl.c0;
  if (r0 >= m) return;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  Acc acc[NP][2][2];
  for (int p = 0; p < NP; ++p)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) acc[p][i][j] = Acc{0, 0, 0, 0};
  // slab j0 of S(R, tau) and Omega(tau, :) in registers (4 + 4 values per thread),
  // prefetched while the previous slab is consumed from LDS
  T sreg[4], oreg[4];
  auto load = [&](int j0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      const int rr = e % 64, kk = e / 64;
      const int r = r0 + rr, jj = j0 + kk;
      sreg[u] = (r < m && jj < h.hi) ? b.S[s_cand[r] + (size_t)jj * n] : traits<T>::zero();
      const int kk2 = e % KC, cc = e / KC;
      const int jj2 = j0 + kk2, c = c0 + cc;
      oreg[u] = (jj2 < h.hi && c < l) ? b.Om[jj2 + (size_t)c * n] : traits<T>::zero();
    }
  };
  load(h.lo);
  for (int j0 = h.lo; j0 < h.hi; j0 += KC) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      const R sr = traits<T>::re(sreg[u]), si = traits<T>::im(sreg[u]);
      const R orr = traits<T>::re(oreg[u]), oi = traits<T>::im(oreg[u]);
      Sg[0][e / 64][e % 64] = sr;
      Og[0][e % KC][e / KC] = orr;
      if constexpr (CX) {
        Sg[1][e / 64][e % 64] = si;
        Og[1][e % KC][e / KC] = oi;
      }
      if constexpr (G3) {
        Sg[2][e / 64][e % 64] = sr + si;
        Og[2][e % KC][e / KC] = orr + oi;
      }
    }
    __syncthreads();
    if (j0 + KC < h.hi) load(j0 + KC);
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      const int kk = ks + lk;
      R a[NP][2], bb[NP][2];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        a[p][0] = Sg[p][kk][wm + li];
        a[p][1] = Sg[p][kk][wm + 16 + li];
        bb[p][0] = Og[p][kk][wn + li];
        bb[p][1] = Og[p][kk][wn + 16 + li];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if constexpr (G3) {
            acc[0][i][j] = mfma_acc<R>::mac(a[0][i], bb[0][j], acc[0][i][j]);
            acc[1][i][j] = mfma_acc<R>::mac(a[1][i], bb[1][j], acc[1][i][j]);
            acc[2][i][j] = mfma_acc<R>::mac(a[2][i], bb[2][j], acc[2][i][j]);
          } else if constexpr (CX) {
            acc[0][i][j] = mfma_acc<R>::mac(a[0][i], bb[0][j], acc[0][i][j]);
            acc[0][i][j] = mfma_acc<R>::mac(-a[1][i], bb[1][j], acc[0][i][j]);
            acc[1][i][j] = mfma_acc<R>::mac(a[0][i], bb[1][j], acc[1][i][j]);
            acc[1][i][j] = mfma_acc<R>::mac(a[1][i], bb[0][j], acc[1][i][j]);
          } else {
            acc[0][i][j] = mfma_acc<R>::mac(a[0][i], bb[0][j], acc[0][i][j]);
          }
        }
    }
  }
  // lane holds column li and four rows of each 16x16 block: Y first for all 16
  // outputs, then the stores (a store the compiler cannot separate from the next
  // load would serialize the read-store pairs)
  T yv[2][2][4];
  static_for<0, 2>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    static_for<0, 2>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      const int c = c0 + wn + 16 * j + li;
      static_for<0, 4>([&](auto vv) {
        constexpr int v = decltype(vv)::value;
        const int r = r0 + wm + 16 * i + mfma_acc<R>::row(lk, v);
        const int row = s_cand[r < m ? r : 0];
        yv[i][j][v] = (r < m && c < l) ? b.Y[row + (size_t)c * n] : traits<T>::zero();
      });
    });
  });
  static_for<0, 2>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    static_for<0, 2>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      const int c = c0 + wn + 16 * j + li;
      static_for<0, 4>([&](auto vv) {
        constexpr int v = decltype(vv)::value;
        const int r = r0 + wm + 16 * i + mfma_acc<R>::row(lk, v);
        if (r < m && c < l) {
          T val;
          if constexpr (G3) {
            const R t0 = acc[0][i][j][v], t1 = acc[1][i][j][v];
            val = traits<T>::mk(t0 - t1, acc[2][i][j][v] - t0 - t1);
          } else if constexpr (CX) {
            val = traits<T>::mk(acc[0][i][j][v], acc[1][i][j][v]);
          } else {
            val = acc[0][i][j][v];
          }
          h.Zt[c + (size_t)r * l] = yv[i][j][v] - val;
        }
      });
    });
  });
  if (tid == 0 && r0 == 0 && c0 == 0) *h.k = m;  // provisional: number of candidates (read by cpqr)
}

// One workgroup per HSS node: truncated CPQR of Zt (l x m) -> k, skeleton, U.
// The working copy sits in LDS when it fits (LDS = true), else in the node's
// global scratch Zw; Zt itself keeps the samples. Columns are never moved: the
// pivot of step j is a physical column chosen from exact trailing norms; every
// wave takes the same decision from the same LDS data (bit-identical butterfly
// reductions), so one barrier per step suffices. Groups of GL lanes apply the
// reflector to one column each and produce that column's trailing norm for the
// next step. Reductions run in the real type of the factor.
//
// Bounded interpolation coefficients (Section 1: no entry of P above 2 in
// modulus): after T = R11^{-1} R12 is formed, while max |T| > 2 the skeleton
// column i and the free column c of the largest |T(i, c)| (ties: lowest i, then
// lowest candidate index c) trade places, the incoming column taking skeleton
// position i, and the QR is redone without pivoting in that column order (a
// strong-RRQR swap with f = 2; each multiplies |det R11| by more than 2, so the
// loop ends; at most kMaxSwaps are taken). k does not change.
//
// GL lanes per column group; each lane holds up to RPL rows of the reflector and
// of the column it updates in registers (GL * RPL >= l). MCAP bounds the number
// of candidates m, KCAP the sample count l (and so the rank).
constexpr int kMaxSwaps = 64;
template <class T, bool LDS, int GL, int RPL, int MCAP, int KCAP, int NT>
__device__ __forceinline__ void cpqr_node(const CompBox<T>* __restrict__ bx, const HssDesc<T>* __restrict__ hs,
                                          int node, int p_os) {
  using R = typename traits<T>::real;
  static_assert(GL * RPL >= KCAP, "reflector rows per group");
  static_assert(MCAP <= 64 * 32, "pivot bit mask");
  const HssDesc<T> h = hs[node];
  const CompBox<T> b = bx[h.box];
  const int l = b.l;
  const int m = *h.k;
  constexpr int NG = NT / GL;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* A = LDS ? (T*)smem_raw : h.Zw;  // l x m, ld = l
  __shared__ R s_nrm[2][MCAP];  // double buffered: read at step j, written for step j + 1
  __shared__ int s_sel[KCAP];
  __shared__ int s_pos[MCAP];   // column -> skeleton position, or -1
  __shared__ T s_rdiag[KCAP];
  __shared__ int s_k;
  __shared__ unsigned s_tm;
  __shared__ unsigned long long s_key;
  const int tid = threadIdx.x, lane = tid & 63;
  const int gid = tid / GL, gl = tid % GL;
  const double thresh = b.tol_scale * sqrt(*b.nrm2) / sqrt(2.0 * (double)max(b.n_id, 1)) * sqrt((double)l);
  const int kcap = min(l, m);
  int k = kcap;
  float tm = 0.f;
  for (int pass = 0, swaps = 0;; ++pass) {
    const bool forced = pass > 0;  // pivot order given by s_sel
    for (int e = tid; e < l * m; e += NT) A[e] = h.Zt[e];
    for (int c = tid; c < m; c += NT) s_pos[c] = -1;
    if (tid == 0) s_tm = 0u;
    __syncthreads();
    for (int c0 = 0; c0 < m; c0 += NG) {
      const int c = c0 + gid;
      R s2 = 0;
      if (c < m)
        for (int r = gl; r < l; r += GL) s2 += traits<T>::abs2(A[r + (size_t)c * l]);
      s2 = group_sum<GL>(s2);
      if (c < m && gl == 0) s_nrm[0][c] = s2;
    }
    __syncthreads();
    unsigned chosen = 0;  // bit t: column lane + 64 t was a pivot (identical in every wave)
    const int jend = forced ? k : kcap;
    for (int j = 0; j < jend; ++j) {
      int p;
      if (!forced) {
        R best = -1, tot = 0;
        int bi = 0x7fffffff;
        for (int t = 0; lane + 64 * t < m; ++t) {
          if ((chosen >> t) & 1u) continue;
          const int c = lane + 64 * t;
          const R v = s_nrm[j & 1][c];
          tot += v;
          if (v > best) {
            best = v;
            bi = c;
          }
        }
        tot = wave_sum(tot);
        wave_argmax(best, bi);
        if (sqrt((double)tot) <= thresh || bi >= m) {
          k = j;
          break;
        }
        p = bi;
        if ((p & 63) == lane) chosen |= 1u << (p >> 6);
        if (tid == 0) s_sel[j] = p;
      } else {
        p = s_sel[j];
      }
      if (tid == 0) s_pos[p] = j;
      // Householder reflector of column p (scalars in the factor's own precision)
      const T x0 = A[j + (size_t)p * l];
      const R xn2 = s_nrm[j & 1][p];
      const R xn = sqrt(xn2);
      const R a0 = sqrt(traits<T>::abs2(x0));
      const R sc = a0 > 0 ? xn / a0 : R(0);
      const T alpha = a0 > 0 ? traits<T>::mk(-traits<T>::re(x0) * sc, -traits<T>::im(x0) * sc)
                             : traits<T>::mk(-xn, 0.0);
      if (tid == 0) s_rdiag[j] = alpha;
      const R vv = R(2) * xn2 + R(2) * a0 * xn;
      const R f = vv > 0 ? R(2) / vv : R(0);
      const T vj = x0 - alpha;
      // this lane's rows r = j + gl + GL t of the reflector, in registers
      T vr[RPL];
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = j + gl + GL * t;
        vr[t] = r < l ? (r == j ? vj : A[r + (size_t)p * l]) : traits<T>::zero();
      }
      const int ncol_iter = (m + NG - 1) / NG;
      for (int it = 0; it < ncol_iter; ++it) {
        const int c = it * NG + gid;
        // earlier pivots are in s_pos (written before the last barrier); p is this step's
        const bool active = c < m && c != p && s_pos[c] < 0;
        T ar[RPL];
        R dre = 0, dim = 0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int r = j + gl + GL * t;
          ar[t] = (active && r < l) ? A[r + (size_t)c * l] : traits<T>::zero();
          const T pr = sc_mul(traits<T>::conj(vr[t]), ar[t]);
          dre += traits<T>::re(pr);
          dim += traits<T>::im(pr);
        }
        dre = group_sum<GL>(dre);
        if (traits<T>::cplx) dim = group_sum<GL>(dim);
        R s2 = 0;
        if (active) {
          const T fw = traits<T>::mk(dre * f, dim * f);
#pragma unroll
          for (int t = 0; t < RPL; ++t) {
            const int r = j + gl + GL * t;
            if (r < l) {
              const T nv = sc_fms(ar[t], fw, vr[t]);
              A[r + (size_t)c * l] = nv;
              if (r > j) s2 += traits<T>::abs2(nv);
            }
          }
        }
        s2 = group_sum<GL>(s2);
        if (active && gl == 0) s_nrm[(j + 1) & 1][c] = s2;
      }
      __syncthreads();
    }
    if (!forced) {
      if (tid == 0) s_k = k;
      __syncthreads();
      k = s_k;
    }
    // T = R11^{-1} R12, one group per free column: back substitution in axpy form
    // (x_i final -> broadcast -> subtract R(0:i, i) x_i); rows are spread over the lanes.
    tm = 0.f;
    for (int c0 = 0; c0 < m; c0 += NG) {
      const int c = c0 + gid;
      const bool act = c < m && s_pos[c] < 0;
      T* col = A + (size_t)(act ? c : 0) * l;
      for (int i = k - 1; i >= 0; --i) {
        const int src = i % GL;
        T xi = traits<T>::zero();
        if (act && gl == src) {
          const T d = s_rdiag[i];
          xi = traits<T>::abs2(d) > 0 ? sc_mul(col[i], sc_inv(d)) : traits<T>::zero();
          col[i] = xi;
          tm = fmaxf(tm, (float)sqrt((double)traits<T>::abs2(xi)));
        }
        const R xr = __shfl(traits<T>::re(xi), src, GL);
        const R xim = __shfl(traits<T>::im(xi), src, GL);
        const T xv = traits<T>::mk(xr, xim);
        if (act)
          for (int r = gl; r < i; r += GL) col[r] = sc_fms(col[r], A[r + (size_t)s_sel[i] * l], xv);
      }
    }
    for (int off = 32; off > 0; off >>= 1) tm = fmaxf(tm, __shfl_xor(tm, off));
    if (lane == 0) atomicMax(&s_tm, __float_as_uint(tm));  // non-negative: bit order = value order
    if (tid == 0) s_key = 0ull;
    __syncthreads();
    tm = __uint_as_float(s_tm);
    if (!(tm > 2.f) || swaps >= kMaxSwaps) break;
    // the swap: largest |T(i, c)|, then the lowest i, then the lowest c
    unsigned long long key = 0ull;
    for (int e = tid; e < k * m; e += NT) {
      const int i = e % k, c = e / k;
      if (s_pos[c] >= 0) continue;
      const float v = (float)sqrt((double)traits<T>::abs2(A[i + (size_t)c * l]));
      const unsigned long long kk = ((unsigned long long)__float_as_uint(v) << 32) |
                                    (unsigned long long)(~(unsigned)(i * MCAP + c));
      key = kk > key ? kk : key;
    }
    atomicMax(&s_key, key);
    __syncthreads();
    if (tid == 0) {
      const unsigned idx = ~(unsigned)(s_key & 0xffffffffull);
      s_sel[idx / MCAP] = (int)(idx % MCAP);
    }
    ++swaps;
    __syncthreads();
  }
  // U (m x k, ld zcap): row sel[i] = e_i, free row c = T(:, c)^T
  for (int e = tid; e < m * k; e += NT) {
    const int c = e % m, i = e / m;
    const int pos = s_pos[c];
    T v;
    if (pos >= 0) v = (pos == i) ? traits<T>::one() : traits<T>::zero();
    else v = A[i + (size_t)c * l];
    h.U[c + (size_t)i * h.zcap] = v;
  }
  for (int i = tid; i < k; i += NT) h.skel[i] = h.cand[s_sel[i]];
  if (tid == 0) atomicMax((int*)b.tmax, __float_as_int(tm));
  __syncthreads();
  if (tid == 0) {
    *h.k = k;
    atomicMax(b.kmax, k);
    if (k < m && k + p_os > l) atomicOr(b.flags, 1);
  }
}

// one workgroup per node of the list
template <class T, bool LDS, int GL, int RPL, int MCAP, int KCAP, int NT = 256>
__global__ __launch_bounds__(NT) void cpqr_kernel(const CompBox<T>* __restrict__ bx,
                                                   const HssDesc<T>* __restrict__ hs,
                                                   const int* __restrict__ list, int p_os) {
  cpqr_node<T, LDS, GL, RPL, MCAP, KCAP, NT>(bx, hs, list[blockIdx.x], p_os);
}

// Persistent form over a work queue: a grid sized to what the chip holds at once
// takes the n nodes of the list in its order (largest first), each workgroup
// claiming the next one from *next (zero at launch) when it finishes the last.
// Every workgroup leaves once the queue is drained.
template <class T, bool LDS, int GL, int RPL, int MCAP, int KCAP>
__global__ __launch_bounds__(256) void cpqr_queue_kernel(const CompBox<T>* __restrict__ bx,
                                                         const HssDesc<T>* __restrict__ hs,
                                                         const int* __restrict__ list, int n, int* __restrict__ next,
                                                         int p_os) {
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(next, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();  // read by every thread before the next claim overwrites it
    if (it >= n) break;
    cpqr_node<T, LDS, GL, RPL, MCAP, KCAP, 256>(bx, hs, list[it], p_os);
    __syncthreads();  // the node's LDS state is dead before the next node's set-up
  }
}

// Tall bases of one HSS height, one workgroup per (HSS node, 64-row tile):
// leaves copy U, parents compute diag(Ut_a, Ut_b) U. Thread = (row, column
// group of 4): each loaded Ut entry is reused for the thread's columns.
template <class T>
__global__ __launch_bounds__(256) void utall_kernel(const CompBox<T>* __restrict__ bx,
                                                    const HssDesc<T>* __restrict__ hs,
                                                    const HTile* __restrict__ tiles) {
  const HTile tl = tiles[blockIdx.x];
  const HssDesc<T> h = hs[tl.hnode];
  const int k = *h.k;
  const int nt = h.hi - h.lo;
  const int rl = threadIdx.x & 63, cg = threadIdx.x >> 6;
  const int r = tl.r0 + rl;
  if (h.left < 0) {
    if (r < nt)
      for (int c0 = cg; c0 < k; c0 += 32) {  // eight loads in flight, then the stores
        T v[8];
        static_for<0, 8>([&](auto tt) {
          constexpr int t = decltype(tt)::value;
          const int c = c0 + 4 * t;
          v[t] = c < k ? h.U[r + (size_t)c * h.zcap] : traits<T>::zero();
        });
        static_for<0, 8>([&](auto tt) {
          constexpr int t = decltype(tt)::value;
          const int c = c0 + 4 * t;
          if (c < k) h.Ut[r + (size_t)c * nt] = v[t];
        });
      }
    return;
  }
  const HssDesc<T> a = hs[h.left], bb = hs[h.right];
  const int ka = *a.k, kb = *bb.k;
  const int na = a.hi - a.lo, nbb = bb.hi - bb.lo;
  if (r >= nt) return;
  const bool left = r < na;
  const T* src = left ? a.Ut + r : bb.Ut + (r - na);
  const int ns = left ? na : nbb;
  const int kk = left ? ka : kb;
  const int qoff = left ? 0 : ka;
  for (int c0 = cg; c0 < k; c0 += 64) {
    T acc[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = traits<T>::zero();
    for (int q = 0; q < kk; ++q) {
      const T u = src[(size_t)q * ns];
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int c = c0 + 4 * t;
        if (c < k) acc[t] = acc[t] + sc_mul(u, h.U[qoff + q + (size_t)c * h.zcap]);
      }
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int c = c0 + 4 * t;
      if (c < k) h.Ut[r + (size_t)c * nt] = acc[t];
    }
  }
}

// S~ off-diagonal blocks of an internal HSS node with children a, c: the block
// Ut_a (S(J_a, J_c) Ut_c^T) and its mirror. Three launches over all internal nodes:
// expand_tmp_kernel forms Et = S(J_a, J_c) Ut_c^T (k_a x n_c), the batched MFMA
// GEMM forms Ut_a Et in place in S~ (its depth k_a is set on the device by
// set_depth_kernel, since the ranks are known there only), and mirror_kernel
// writes the transposed block.

// Et, one workgroup per (internal node, 64 x 64 tile of Et); each thread 4 x 4 values
template <class T>
__global__ __launch_bounds__(256) void expand_tmp_kernel(const CompBox<T>* __restrict__ bx,
                                                         const HssDesc<T>* __restrict__ hs,
                                                         const HTile* __restrict__ tiles) {
  const HTile tl = tiles[blockIdx.x];
  const HssDesc<T> h = hs[tl.hnode];
  const HssDesc<T> a = hs[h.left], c = hs[h.right];
  const int ka = *a.k, kc = *c.k;
  if (tl.r0 >= ka) return;
  const CompBox<T> b = bx[h.box];
  const int nc = c.hi - c.lo, n = b.n;
  __shared__ T Gs[16][65];  // S(J_a, J_c) slab: 16 skeleton columns of c x 64 rows
  __shared__ T Us[16][65];  // Ut_c^T slab: 16 ranks x 64 columns
  __shared__ int s_ra[64];
  const int tid = threadIdx.x, ti = tid & 15, tj = tid >> 4;
  if (tid < 64) s_ra[tid] = tl.r0 + tid < ka ? a.skel[tl.r0 + tid] : 0;
  T acc[4][4];
  static_for<0, 4>([&](auto uu) {
    static_for<0, 4>([&](auto vv) { acc[decltype(uu)::value][decltype(vv)::value] = traits<T>::zero(); });
  });
  __syncthreads();
  for (int q0 = 0; q0 < kc; q0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int qq = e >> 6, i = e & 63, q = q0 + qq;
      const bool in = q < kc && tl.r0 + i < ka;
      Gs[qq][i] = in ? b.S[s_ra[i] + (size_t)c.skel[in ? q : 0] * n] : traits<T>::zero();
      const bool inu = q < kc && tl.c0 + i < nc;
      Us[qq][i] = inu ? c.Ut[(tl.c0 + i) + (size_t)(inu ? q : 0) * nc] : traits<T>::zero();
    }
    __syncthreads();
#pragma unroll 4
    for (int qq = 0; qq < 16; ++qq) {
      T g[4], u[4];
      static_for<0, 4>([&](auto xx) {
        constexpr int x = decltype(xx)::value;
        g[x] = Gs[qq][ti + 16 * x];
        u[x] = Us[qq][tj + 16 * x];
      });
      static_for<0, 4>([&](auto uu) {
        static_for<0, 4>([&](auto vv) {
          constexpr int x = decltype(uu)::value, y = decltype(vv)::value;
          acc[x][y] = acc[x][y] + sc_mul(g[x], u[y]);
        });
      });
    }
    __syncthreads();
  }
  static_for<0, 4>([&](auto uu) {
    static_for<0, 4>([&](auto vv) {
      constexpr int x = decltype(uu)::value, y = decltype(vv)::value;
      const int r = tl.r0 + ti + 16 * x, col = tl.c0 + tj + 16 * y;
      if (r < ka && col < nc) h.Et[r + (size_t)col * h.ldet] = acc[x][y];
    });
  });
}

// the depth of every expand GEMM: D[i].K = *kp[i]
template <class D>
__global__ void set_depth_kernel(D* __restrict__ d, const int* const* __restrict__ kp, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i].K = *kp[i];
}

// S~(J_c-range, J_a-range) = S~(J_a-range, J_c-range)^T through an LDS tile; one
// workgroup per (internal node, MT x MT tile of the a x c block)
template <class T, int MT>
__global__ __launch_bounds__(256) void mirror_kernel(const CompBox<T>* __restrict__ bx,
                                                     const HssDesc<T>* __restrict__ hs,
                                                     const HTile* __restrict__ tiles) {
  const HTile tl = tiles[blockIdx.x];
  const HssDesc<T> h = hs[tl.hnode];
  const CompBox<T> b = bx[h.box];
  const HssDesc<T> a = hs[h.left], c = hs[h.right];
  const int na = a.hi - a.lo, nc = c.hi - c.lo, n = b.n;
  __shared__ T t[MT][MT + 1];
  for (int e = threadIdx.x; e < MT * MT; e += 256) {
    const int i = e % MT, j = e / MT;
    if (tl.r0 + i < na && tl.c0 + j < nc) t[j][i] = b.St[(a.lo + tl.r0 + i) + (size_t)(c.lo + tl.c0 + j) * n];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < MT * MT; e += 256) {
    const int j = e % MT, i = e / MT;
    if (tl.r0 + i < na && tl.c0 + j < nc) b.St[(c.lo + tl.c0 + j) + (size_t)(a.lo + tl.r0 + i) * n] = t[j][i];
  }
}

// copy of the HSS leaf diagonal blocks; grid: one workgroup per HSS leaf
template <class T>
__global__ __launch_bounds__(256) void diag_copy_kernel(const CompBox<T>* __restrict__ bx,
                                                        const HssDesc<T>* __restrict__ hs,
                                                        const int* __restrict__ list) {
  const HssDesc<T> h = hs[list[blockIdx.x]];
  const CompBox<T> b = bx[h.box];
  const int nt = h.hi - h.lo;
  for (int e = threadIdx.x; e < nt * nt; e += 256) {
    const int r = h.lo + e % nt, c = h.lo + e / nt;
    b.St[r + (size_t)c * b.n] = b.S[r + (size_t)c * b.n];
  }
}

// grid (chunks, boxes): ||S - S~||_F^2
template <class T>
__global__ __launch_bounds__(256) void judge_kernel(const CompBox<T>* __restrict__ bx) {
  const CompBox<T> b = bx[blockIdx.y];
  const int64_t tot = (int64_t)b.n * b.n;
  double acc = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256)
    acc += (double)traits<T>::abs2(b.S[e] - b.St[e]);
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(b.err2, red[0]);
}

// grid (chunks, boxes): S~ = S (tol = 0 or fallback)
template <class T>
__global__ void copy_box_kernel(const CompBox<T>* __restrict__ bx) {
  const CompBox<T> b = bx[blockIdx.y];
  const int64_t tot = (int64_t)b.n * b.n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256)
    b.St[e] = b.S[e];
}

}  // namespace hss
