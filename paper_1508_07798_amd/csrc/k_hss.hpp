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
  double tol_scale;  // tol * 2^-(2 * retries)
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
  T* Zt;              // l x zcap workspace (samples, then QR)
  T* U;               // zcap x l interpolation matrix (ld = zcap)
  T* Ut;              // (hi - lo) x l tall basis (ld = hi - lo)
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

// grid (chunks, boxes): S <- (S + S^T)/2 and ||S||_F^2 (atomic partial sums)
template <class T>
__global__ __launch_bounds__(256) void symm_norm_kernel(const CompBox<T>* __restrict__ bx) {
  const CompBox<T> b = bx[blockIdx.y];
  const int64_t tot = (int64_t)b.n * b.n;
  double acc = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int r = (int)(e % b.n), c = (int)(e / b.n);
    if (r < c) {
      T* a = b.S + r + (size_t)c * b.n;
      T* t = b.S + c + (size_t)r * b.n;
      T m = traits<T>::mk(0.5 * (traits<T>::re(*a) + traits<T>::re(*t)),
                          0.5 * (traits<T>::im(*a) + traits<T>::im(*t)));
      *a = m;
      *t = m;
      acc += 2.0 * (double)traits<T>::abs2(m);
    } else if (r == c) {
      acc += (double)traits<T>::abs2(b.S[e]);
    }
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

// one workgroup per HSS node of one height: candidates and samples
template <class T>
__global__ __launch_bounds__(256) void sample_kernel(const CompBox<T>* __restrict__ bx,
                                                     const HssDesc<T>* __restrict__ hs,
                                                     const int* __restrict__ list) {
  const HssDesc<T> h = hs[list[blockIdx.x]];
  const CompBox<T> b = bx[h.box];
  __shared__ int s_cand[512];
  __shared__ int s_m;
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
  for (int i = tid; i < m; i += 256) h.cand[i] = s_cand[i];
  const int l = b.l, n = b.n;
  // Zt (l x m, column r = samples of candidate r)
  for (int e = tid; e < m * l; e += 256) {
    const int r = e % m, c = e / m;
    const int row = s_cand[r];
    T acc = b.Y[row + (size_t)c * n];
    for (int j = h.lo; j < h.hi; ++j) acc = sc_fms(acc, b.S[row + (size_t)j * n], b.Om[j + (size_t)c * n]);
    h.Zt[c + (size_t)r * l] = acc;
  }
  if (tid == 0) *h.k = m;  // provisional: number of candidates (read by cpqr)
}

// one workgroup per HSS node: truncated CPQR of Zt (l x m) -> k, skeleton, U
template <class T>
__global__ __launch_bounds__(256) void cpqr_kernel(const CompBox<T>* __restrict__ bx,
                                                   const HssDesc<T>* __restrict__ hs,
                                                   const int* __restrict__ list, double tol,
                                                   int p_os) {
  using R = typename traits<T>::real;
  const HssDesc<T> h = hs[list[blockIdx.x]];
  const CompBox<T> b = bx[h.box];
  const int l = b.l;
  const int m = *h.k;
  T* A = h.Zt;  // l x m, ld = l
  __shared__ double s_nrm[512];
  __shared__ int s_perm[512];
  __shared__ T s_v[256];
  __shared__ double red[256];
  __shared__ int s_k, s_p;
  __shared__ double s_tot;
  const int tid = threadIdx.x;
  const double thresh = b.tol_scale * sqrt(*b.nrm2) / sqrt(2.0 * (double)max(b.n_id, 1)) *
                        sqrt((double)l);
  for (int i = tid; i < m; i += 256) s_perm[i] = i;
  const int kcap = min(l, m);
  int k = kcap;
  __syncthreads();
  for (int j = 0; j < kcap; ++j) {
    // exact norms of the remaining columns over rows j..l-1
    for (int c = j + tid; c < m; c += 256) {
      double s = 0;
      const T* col = A + (size_t)c * l;
      for (int r = j; r < l; ++r) s += (double)traits<T>::abs2(col[r]);
      s_nrm[c] = s;
    }
    __syncthreads();
    if (tid == 0) {
      double tot = 0, best = -1;
      int bi = j;
      for (int c = j; c < m; ++c) {
        tot += s_nrm[c];
        if (s_nrm[c] > best) {
          best = s_nrm[c];
          bi = c;
        }
      }
      s_tot = tot;
      s_p = bi;
    }
    __syncthreads();
    if (sqrt(s_tot) <= thresh) {
      k = j;
      break;
    }
    const int p = s_p;
    if (p != j) {
      for (int r = tid; r < l; r += 256) {
        T t = A[r + (size_t)j * l];
        A[r + (size_t)j * l] = A[r + (size_t)p * l];
        A[r + (size_t)p * l] = t;
      }
      if (tid == 0) {
        int t = s_perm[j];
        s_perm[j] = s_perm[p];
        s_perm[p] = t;
      }
    }
    __syncthreads();
    // Householder vector of A(j:l, j)
    const T x0 = A[j + (size_t)j * l];
    const double xn2 = s_nrm[p];
    const double xn = sqrt(xn2);
    const double a0 = sqrt((double)traits<T>::abs2(x0));
    // alpha = -(x0/|x0|) ||x||
    T alpha;
    if (a0 > 0) alpha = traits<T>::mk(-traits<T>::re(x0) / a0 * xn, -traits<T>::im(x0) / a0 * xn);
    else alpha = traits<T>::mk(-xn, 0.0);
    const double vv = 2.0 * xn2 + 2.0 * a0 * xn;  // ||x - alpha e1||^2
    for (int r = j + tid; r < l; r += 256) {
      T v = A[r + (size_t)j * l];
      if (r == j) v = v - alpha;
      s_v[r - j] = v;
    }
    __syncthreads();
    if (vv > 0) {
      for (int c = j + 1 + tid; c < m; c += 256) {
        T* col = A + (size_t)c * l;
        T w = traits<T>::zero();
        for (int r = j; r < l; ++r) w = w + sc_mul(traits<T>::conj(s_v[r - j]), col[r]);
        const double f = 2.0 / vv;
        const T fw = traits<T>::mk(traits<T>::re(w) * f, traits<T>::im(w) * f);
        for (int r = j; r < l; ++r) col[r] = sc_fms(col[r], fw, s_v[r - j]);
      }
    }
    __syncthreads();
    if (tid == 0) {
      A[j + (size_t)j * l] = alpha;
      for (int r = j + 1; r < l; ++r) A[r + (size_t)j * l] = traits<T>::zero();
    }
    __syncthreads();
  }
  if (tid == 0) s_k = k;
  __syncthreads();
  k = s_k;
  // T = R11^{-1} R12 in place (columns k..m-1, rows 0..k-1), one column per thread
  float tm = 0.f;
  for (int c = k + tid; c < m; c += 256) {
    T* col = A + (size_t)c * l;
    for (int i = k - 1; i >= 0; --i) {
      T x = col[i];
      for (int jj = i + 1; jj < k; ++jj) x = sc_fms(x, A[i + (size_t)jj * l], col[jj]);
      const T d = A[i + (size_t)i * l];
      x = traits<T>::abs2(d) > 0 ? sc_mul(x, sc_inv(d)) : traits<T>::zero();
      col[i] = x;
      tm = fmaxf(tm, (float)sqrt((double)traits<T>::abs2(x)));
    }
  }
  __syncthreads();
  // U (m x k, ld zcap): rows perm[0..k) = I, rows perm[k..m) = T^T
  for (int e = tid; e < m * k; e += 256) {
    const int r = e % m, c = e / m;  // r: position in pivot order
    T v;
    if (r < k) v = (r == c) ? traits<T>::one() : traits<T>::zero();
    else v = A[c + (size_t)r * l];
    h.U[s_perm[r] + (size_t)c * h.zcap] = v;
  }
  for (int i = tid; i < k; i += 256) h.skel[i] = h.cand[s_perm[i]];
  // stats
  for (int off = 32; off > 0; off >>= 1) tm = fmaxf(tm, __shfl_xor(tm, off));
  if ((tid & 63) == 0) atomicMax((int*)b.tmax, __float_as_int(tm));
  if (tid == 0) {
    *h.k = k;
    atomicMax(b.kmax, k);
    if (k < m && k + p_os > l) atomicOr(b.flags, 1);
  }
}

// tall bases of one HSS height: leaves copy U, parents diag(Ut_a, Ut_b) U
template <class T>
__global__ __launch_bounds__(256) void utall_kernel(const CompBox<T>* __restrict__ bx,
                                                    const HssDesc<T>* __restrict__ hs,
                                                    const int* __restrict__ list) {
  const HssDesc<T> h = hs[list[blockIdx.x]];
  const int k = *h.k;
  const int nt = h.hi - h.lo;
  if (h.left < 0) {
    for (int e = threadIdx.x; e < nt * k; e += 256) {
      const int r = e % nt, c = e / nt;
      h.Ut[r + (size_t)c * nt] = h.U[r + (size_t)c * h.zcap];
    }
    return;
  }
  const HssDesc<T> a = hs[h.left], bb = hs[h.right];
  const int ka = *a.k, kb = *bb.k;
  const int na = a.hi - a.lo, nbb = bb.hi - bb.lo;
  for (int e = threadIdx.x; e < nt * k; e += 256) {
    const int r = e % nt, c = e / nt;
    T acc = traits<T>::zero();
    if (r < na) {
      for (int q = 0; q < ka; ++q) acc = acc + sc_mul(a.Ut[r + (size_t)q * na], h.U[q + (size_t)c * h.zcap]);
    } else {
      const int rr = r - na;
      for (int q = 0; q < kb; ++q)
        acc = acc + sc_mul(bb.Ut[rr + (size_t)q * nbb], h.U[ka + q + (size_t)c * h.zcap]);
    }
    h.Ut[r + (size_t)c * nt] = acc;
  }
}

// S~ off-diagonal blocks. One workgroup per (internal HSS node, tw-column tile of its
// right child): out(:, tile) = Ut_a * (S(J_a, J_b) * Ut_b(tile, :)^T), mirrored.
struct ExpandTile {
  int hnode;   // internal HSS node
  int c0;      // first column (within the right child) of the tile
};
template <class T>
__global__ __launch_bounds__(256) void expand_kernel(const CompBox<T>* __restrict__ bx,
                                                     const HssDesc<T>* __restrict__ hs,
                                                     const ExpandTile* __restrict__ tiles, int tw) {
  const ExpandTile tl = tiles[blockIdx.x];
  const HssDesc<T> h = hs[tl.hnode];
  const CompBox<T> b = bx[h.box];
  const HssDesc<T> a = hs[h.left], c = hs[h.right];
  const int ka = *a.k, kc = *c.k;
  const int na = a.hi - a.lo, nc = c.hi - c.lo;
  const int cw = min(tw, nc - tl.c0);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tmp = (T*)smem_raw;  // ka x tw
  const int n = b.n;
  for (int e = threadIdx.x; e < ka * cw; e += 256) {
    const int i = e % ka, j = e / ka;
    const int si = a.skel[i];
    T acc = traits<T>::zero();
    for (int q = 0; q < kc; ++q)
      acc = acc + sc_mul(b.S[si + (size_t)c.skel[q] * n], c.Ut[(tl.c0 + j) + (size_t)q * nc]);
    tmp[i + j * ka] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < na * cw; e += 256) {
    const int r = e % na, j = e / na;
    T acc = traits<T>::zero();
    for (int q = 0; q < ka; ++q) acc = acc + sc_mul(a.Ut[r + (size_t)q * na], tmp[q + j * ka]);
    const int gr = a.lo + r, gc = c.lo + tl.c0 + j;
    b.St[gr + (size_t)gc * n] = acc;
    b.St[gc + (size_t)gr * n] = acc;
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
