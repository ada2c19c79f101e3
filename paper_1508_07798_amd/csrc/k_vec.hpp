// Vector kernels: the sweeps of the inverse factorization, the element-block
// SpMV and the GMRES building blocks. Vectors are FP64 (complex128); stored
// factors may be FP32 and are widened on load.
#pragma once

#include "common.hpp"

namespace hss {

// Batched GEMV y(out) = or -= Mat * x(in) on multi-vectors (nrhs columns, ld).
// Rows / columns are either contiguous from an offset or listed by index.
template <class T> struct GemvDesc {
  const T* mat;          // rows x cols, column-major, ld = ldm (rows when ldm is 0)
  int rows, cols;
  int64_t in_off;        // contiguous input offset, or -1 to use in_idx
  const int64_t* in_idx;
  int64_t out_off;       // contiguous output offset, or -1 to use out_idx
  const int64_t* out_idx;
  const int* in_perm;    // if set: input c is in_off + in_perm[c] (a permuted contiguous segment)
  int ldm;               // leading dimension of mat (0: rows)
};

// Work item of a GEMV launch: rows [r0, r0 + 64) and columns [c0, c1) of entry
// `entry`; split != 0 when the entry's columns are spread over several items,
// whose partial sums are then combined with atomic adds.
struct GemvTile {
  int entry, r0, c0, c1, split;
};

template <class V> __device__ __forceinline__ void atomic_add_v(V* p, V v);
template <> __device__ __forceinline__ void atomic_add_v<double>(double* p, double v) { atomicAdd(p, v); }
template <> __device__ __forceinline__ void atomic_add_v<cd>(cd* p, cd v) {
  atomicAdd(&p->x, v.x);
  atomicAdd(&p->y, v.y);
}

// sub = 0: y = M x (outputs of split entries must be zero beforehand); sub = 1:
// y -= M x; sub = 2: y += M x. One workgroup per tile: 512 threads = 64 rows x 8
// column groups, matrix loads four at a time, x staged through LDS in chunks of
// 256 columns.
constexpr int GEMV_THREADS = 512;
template <class T, class V, int NR>
__global__ __launch_bounds__(GEMV_THREADS) void gemv_kernel(const GemvDesc<T>* __restrict__ ds,
                                                            const GemvTile* __restrict__ tiles,
                                                            const V* __restrict__ x, V* __restrict__ y,
                                                            int64_t ld, int nrhs, int sub) {
  constexpr int NP = GEMV_THREADS / 64;
  const GemvTile tl = tiles[blockIdx.x];
  const GemvDesc<T> d = ds[tl.entry];
  const int r0 = tl.r0;
  const int tid = threadIdx.x;
  const int rl = tid & 63, part = tid >> 6;
  const int row = r0 + rl;
  __shared__ V xs[NR][256];
  __shared__ V red[NP][64];  // one right-hand side at a time: four workgroups fit a CU
  for (int rb = 0; rb < nrhs; rb += NR) {
    const int nr = min(NR, nrhs - rb);
    V acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = traits<V>::zero();
    for (int c0 = tl.c0; c0 < tl.c1; c0 += 256) {
      const int cw = min(256, tl.c1 - c0);
      __syncthreads();
      for (int e = tid; e < cw * nr; e += GEMV_THREADS) {
        const int c = e % cw, k = e / cw;
        const int64_t src = d.in_perm ? d.in_off + d.in_perm[c0 + c]
                                      : d.in_off >= 0 ? d.in_off + c0 + c : d.in_idx[c0 + c];
        xs[k][c] = x[src + (rb + k) * ld];
      }
      __syncthreads();
      if (row < d.rows) {
        const size_t ldm = d.ldm > 0 ? (size_t)d.ldm : (size_t)d.rows;
        const T* mp = d.mat + row + (size_t)c0 * ldm;
        int c = part;
        for (; c + 3 * NP < cw; c += 4 * NP) {
          T m4[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) m4[u] = mp[(size_t)(c + u * NP) * ldm];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const V mv = to_wide(m4[u]);
#pragma unroll
            for (int k = 0; k < NR; ++k)
              if (k < nr) acc[k] = acc[k] + sc_mul(mv, xs[k][c + u * NP]);
          }
        }
        for (; c < cw; c += NP) {
          const V mv = to_wide(mp[(size_t)c * ldm]);
#pragma unroll
          for (int k = 0; k < NR; ++k)
            if (k < nr) acc[k] = acc[k] + sc_mul(mv, xs[k][c]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if (k >= nr) break;  // nr is the same for the whole workgroup
      red[part][rl] = acc[k];
      __syncthreads();
      if (part == 0 && row < d.rows) {
        const int64_t dst = d.out_off >= 0 ? d.out_off + row : d.out_idx[row];
        V s = red[0][rl];
        for (int q = 1; q < NP; ++q) s = s + red[q][rl];
        V* yp = y + dst + (rb + k) * ld;
        if (tl.split) atomic_add_v(yp, sub == 1 ? -s : s);
        else *yp = sub == 1 ? (*yp - s) : sub == 2 ? (*yp + s) : s;
      }
      __syncthreads();
    }
  }
}

// y[out_off + i] = x[in_off + perm[i]] (x[in_off + i] when perm is null), i < n, for
// every segment and right-hand side; grid (chunks, segments)
struct PermSeg {
  int64_t in_off, out_off;
  const int* perm;
  int n;
};
template <class V>
__global__ void perm_gather_kernel(const V* __restrict__ x, V* __restrict__ y, int64_t ld, int nrhs,
                                   const PermSeg* __restrict__ segs) {
  const PermSeg sg = segs[blockIdx.y];
  const int64_t tot = (int64_t)sg.n * nrhs;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e % sg.n);
    const int64_t k = e / sg.n;
    y[sg.out_off + i + k * ld] = x[sg.in_off + (sg.perm ? sg.perm[i] : i) + k * ld];
  }
}

// zero y over contiguous segments (off[i], len[i]) for all nrhs columns; a kernel,
// not a memset, because the sweeps are captured into a graph
template <class V>
__global__ void zero_segments_kernel(V* __restrict__ y, int64_t ld, int nrhs, const int64_t* __restrict__ off,
                                     const int* __restrict__ len, int nseg) {
  const int sgm = blockIdx.y;
  if (sgm >= nseg) return;
  const int64_t o = off[sgm];
  const int n = len[sgm];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)n * nrhs; e += (int64_t)gridDim.x * 256)
    y[o + e % n + (e / n) * ld] = traits<V>::zero();
}

// log10 of the Frobenius norm of every element's diagonal block (rank-model
// features): out[e] = 0.5 log10(sum |A_ee|^2), blk[e] the block index (or -1).
template <class V>
__global__ void diag_lognorm_kernel(const V* __restrict__ vals, const int64_t* __restrict__ blk, int q2, int n,
                                    float* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t b = blk[e];
  double f = 0;
  if (b >= 0)
    for (int k = 0; k < q2; ++k) f += traits<V>::abs2(vals[b * q2 + k]);
  out[e] = (float)(0.5 * log10(f > 1e-300 ? f : 1e-300));
}

// tree order <-> dof order. perm[t] = global dof of tree position t.
template <class V>
__global__ void permute_kernel(const V* __restrict__ x, int64_t ldx, V* __restrict__ y, int64_t ldy,
                               const int64_t* __restrict__ perm, int64_t n, int nrhs, int inverse) {
  const int64_t tot = n * nrhs;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int64_t t = e % n;
    const int64_t k = e / n;
    if (!inverse) y[t + k * ldy] = x[perm[t] + k * ldx];
    else y[perm[t] + k * ldy] = x[t + k * ldx];
  }
}

// dst = src converted elementwise between scalar types (a complex64 block widened
// to complex128 and back)
template <class D, class S>
__global__ __launch_bounds__(256) void convert_kernel(const S* __restrict__ src, D* __restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    dst[e] = traits<D>::mk(traits<S>::re(src[e]), traits<S>::im(src[e]));
}

// dst = src converted for every segment (n elements each); grid (chunks, segments)
template <class D, class S> struct CvtSeg {
  D* dst;
  const S* src;
  int64_t n;
};
template <class D, class S>
__global__ __launch_bounds__(256) void convert_segs_kernel(const CvtSeg<D, S>* __restrict__ segs) {
  const CvtSeg<D, S> sg = segs[blockIdx.y];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < sg.n; e += (int64_t)gridDim.x * 256)
    sg.dst[e] = traits<D>::mk(traits<S>::re(sg.src[e]), traits<S>::im(sg.src[e]));
}

// y = A x (mode 0) or y = b - A x (mode 1) for the element-block operator.
// dof_elem[d]: global element of global dof d; elem_dof[e]: first global dof of e.
template <class V>
__global__ __launch_bounds__(256) void spmv_kernel(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                                                   const V* __restrict__ vals, int q,
                                                   const int32_t* __restrict__ dof_elem,
                                                   const int64_t* __restrict__ elem_dof, int64_t n,
                                                   const V* __restrict__ x, const V* __restrict__ b,
                                                   V* __restrict__ y, int64_t ld, int nrhs, int mode) {
  const int64_t tot = n * nrhs;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int64_t d = e % n, k = e / n;
    const int el = dof_elem[d];
    const int r = (int)(d - elem_dof[el]);
    V acc = traits<V>::zero();
    for (int bb = row_ptr[el]; bb < row_ptr[el + 1]; ++bb) {
      const V* blk = vals + (size_t)bb * q * q + r;
      const V* xs = x + elem_dof[col_idx[bb]] + k * ld;
      for (int c = 0; c < q; ++c) acc = acc + sc_mul(blk[(size_t)c * q], xs[c]);
    }
    y[d + k * ld] = mode == 0 ? acc : (b[d + k * ld] - acc);
  }
}

// ------------------------------------------------------------- GMRES pieces
// Systems s = (problem p, column k): segment [seg_off[p], seg_off[p+1]) of column k.
// Partial sums of conj(V_i) . w over chunks; grid (chunks, systems).
template <class V>
__global__ __launch_bounds__(256) void dots_kernel(const V* __restrict__ Vb, int64_t vstride, int nvec,
                                                   const V* __restrict__ w, int64_t ld,
                                                   const int64_t* __restrict__ seg_off, int nprob,
                                                   int chunk, V* __restrict__ part, int nchunk_max) {
  const int s = blockIdx.y;
  const int p = s % nprob, k = s / nprob;
  const int64_t a = seg_off[p], e = seg_off[p + 1];
  const int64_t c0 = a + (int64_t)blockIdx.x * chunk;
  __shared__ V red[256];
  for (int i = 0; i < nvec; ++i) {
    V acc = traits<V>::zero();
    if (c0 < e) {
      const int64_t c1 = min(e, c0 + chunk);
      const V* vi = Vb + i * vstride + k * ld;
      const V* wk = w + k * ld;
      for (int64_t t = c0 + threadIdx.x; t < c1; t += 256) acc = acc + sc_mul(traits<V>::conj(vi[t]), wk[t]);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[((size_t)s * nchunk_max + blockIdx.x) * nvec + i] = red[0];
    __syncthreads();
  }
}

// out[s * ostride + i] (+)= sum over chunks of part; one thread per (i, s).
template <class V>
__global__ void dots_reduce_kernel(const V* __restrict__ part, int nvec, int nsys, int nchunk_max,
                                   V* __restrict__ out, int ostride, int accumulate) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nvec * nsys) return;
  const int i = t % nvec, s = t / nvec;
  V acc = traits<V>::zero();
  for (int c = 0; c < nchunk_max; ++c) acc = acc + part[((size_t)s * nchunk_max + c) * nvec + i];
  out[(size_t)s * ostride + i] = accumulate ? out[(size_t)s * ostride + i] + acc : acc;
}

// w[:, seg s] = sign * sum_i coef[s*cstride + i] V_i  (+ w if accumulate)
template <class V>
__global__ void combine_kernel(const V* __restrict__ Vb, int64_t vstride, int nvec,
                               const V* __restrict__ coef, int cstride, const int32_t* __restrict__ dof_prob,
                               int nprob, V* __restrict__ w, int64_t ld, int64_t n, int nrhs,
                               double sign, int accumulate) {
  const int64_t tot = n * nrhs;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int64_t d = e % n, k = e / n;
    const int s = dof_prob[d] + (int)k * nprob;
    V acc = traits<V>::zero();
    for (int i = 0; i < nvec; ++i) acc = acc + sc_mul(coef[(size_t)s * cstride + i], Vb[i * vstride + d + k * ld]);
    V* wp = w + d + k * ld;
    V val = sign * acc;
    *wp = accumulate ? (*wp + val) : val;
  }
}

// w[:, seg s] *= scale[s] (scale given as 1/norm with a zero guard)
template <class V>
__global__ void scale_kernel(V* __restrict__ w, int64_t ld, int64_t n, int nrhs, const double* __restrict__ nrm,
                             const int32_t* __restrict__ dof_prob, int nprob, V* __restrict__ dst) {
  const int64_t tot = n * nrhs;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int64_t d = e % n, k = e / n;
    const int s = dof_prob[d] + (int)k * nprob;
    const double v = nrm[s];
    const double f = v > 0 ? 1.0 / v : 0.0;
    dst[d + k * ld] = f * w[d + k * ld];
  }
}

// nrm[s] = sqrt(max(0, re(dot[s]))): the norms that scale_kernel divides by, kept on
// the device (the host reads them later with the Hessenberg column)
template <class V>
__global__ void norm_finish_kernel(const V* __restrict__ dot, double* __restrict__ nrm, int ns) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s < ns) nrm[s] = sqrt(fmax(0.0, (double)traits<V>::re(dot[s])));
}

}  // namespace hss
