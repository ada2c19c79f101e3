// Formation of the dense blocks of every box of a wave.
//
// Leaves (Section 3.1, the sub-matrices of A listed before equation (30)):
//   A^_ii = A(I, I), A^_ib = A(I, B), A^_bi = A(B, I), A^_bb = A(B, B),
// read from the element blocks. Merge boxes (the 2 x 2 block matrices before
// equation (32)): entries whose row and column come from the same child are
// read from that child's compressed complement S~, the others from the
// coupling blocks A(B^mu, B^nu). The root (equation (36)) is a merge with
// I^ = B^2 u B^3 and no B, assembled in FP64.
//
// Outputs per box: M = [A^_ii | A^_ib] (n_i x (n_i + n_b)), A^_bi (n_b x n_i),
// S = A^_bb (n_b x n_b); all column-major.
#pragma once

#include "common.hpp"

namespace hss {

struct OpDev {                // the FP64 operator on the device (all problems)
  const int32_t* row_ptr;     // global element rows
  const int32_t* col_idx;     // global element ids
  const void* vals;           // double / cd, q*q per block, column-major
  int q;
};

template <class TS> struct GatherDesc {
  int ni, nb;
  const int64_t* gidx;     // [ni + nb]: global dofs of I^ then B (problem offset included)
  const int32_t* src;      // merge: [ni + nb] side*2^30 + position in the child's B; null for leaves
  const TS* st[2];         // children's S~ (merge)
  int nbc[2];              // children's B sizes
  int64_t el_off, dof_off; // problem offsets
};

// One workgroup per 64 x 32 tile of a box's (n_i + n_b)^2 entries: the sources of
// the tile's rows and columns (child side and position in its B, global element
// and local dof) are decoded once into LDS, and each thread, which keeps one row,
// looks up the element block of its operator entries once per run of columns of
// the same element (entry (r, c) of block (e, f) sits at c q + r, column-major).
// grid: (tiles of the largest box, boxes).
constexpr int GT_R = 64, GT_C = 32;
template <class T, class TA, class TS>
__global__ __launch_bounds__(256) void gather_tile_kernel(OpDev A, const GatherDesc<TS>* __restrict__ descs,
                                                          T* const* __restrict__ Mout,
                                                          T* const* __restrict__ Abi_out,
                                                          T* const* __restrict__ S_out) {
  const GatherDesc<TS> g = descs[blockIdx.y];
  const int n = g.ni + g.nb;
  const int trows = (n + GT_R - 1) / GT_R, tcols = (n + GT_C - 1) / GT_C;
  if ((int)blockIdx.x >= trows * tcols) return;  // the whole workgroup
  const int r0 = ((int)blockIdx.x % trows) * GT_R, c0 = ((int)blockIdx.x / trows) * GT_C;
  __shared__ int s_side[GT_R + GT_C], s_pos[GT_R + GT_C], s_loc[GT_R + GT_C];
  __shared__ int64_t s_el[GT_R + GT_C];
  const int tid = threadIdx.x, q = A.q;
  if (tid < GT_R + GT_C) {
    // slots 0 .. GT_R - 1: rows r0 + tid; then columns c0 + (tid - GT_R); past the
    // box's end a slot repeats its last index (never used)
    const int i = tid < GT_R ? min(r0 + tid, n - 1) : min(c0 + tid - GT_R, n - 1);
    const int64_t l = g.gidx[i] - g.dof_off;
    s_el[tid] = g.el_off + l / q;
    s_loc[tid] = (int)(l % q);
    if (g.src) {
      const int32_t sv = g.src[i];
      s_side[tid] = sv >> 30;
      s_pos[tid] = sv & ((1 << 30) - 1);
    } else {
      s_side[tid] = -1;
      s_pos[tid] = 0;
    }
  }
  __syncthreads();
  const int rl = tid % GT_R, cg = tid / GT_R;
  const int r = r0 + rl;
  if (r >= n) return;
  T* M = Mout[blockIdx.y];
  T* Abi = Abi_out ? Abi_out[blockIdx.y] : nullptr;
  T* S = S_out ? S_out[blockIdx.y] : nullptr;
  const int side_r = s_side[rl], pos_r = s_pos[rl], loc_r = s_loc[rl];
  const int64_t er = s_el[rl];
  int64_t last_ec = -1;
  int blk = -1;
  for (int cc = cg; cc < GT_C; cc += 256 / GT_R) {
    const int c = c0 + cc;
    if (c >= n) break;
    const int sl = GT_R + cc;
    T v;
    if (side_r >= 0 && side_r == s_side[sl]) {
      const TS* st = g.st[side_r];
      const TS sv = st[pos_r + (size_t)s_pos[sl] * g.nbc[side_r]];
      if constexpr (sizeof(T) == sizeof(TS)) v = sv;
      else v = narrow<T>(to_wide(sv));
    } else {
      const int64_t ec = s_el[sl];
      if (ec != last_ec) {
        last_ec = ec;
        blk = -1;
        for (int b = A.row_ptr[er]; b < A.row_ptr[er + 1]; ++b)
          if (A.col_idx[b] == ec) {
            blk = b;
            break;
          }
      }
      v = blk >= 0 ? narrow<T>(((const TA*)A.vals)[(size_t)blk * q * q + (size_t)s_loc[sl] * q + loc_r])
                   : traits<T>::zero();
    }
    if (r < g.ni) {
      M[r + (size_t)c * g.ni] = v;  // [A_ii | A_ib]
    } else if (c < g.ni) {
      Abi[(r - g.ni) + (size_t)c * g.nb] = v;
    } else {
      S[(r - g.ni) + (size_t)(c - g.ni) * g.nb] = v;
    }
  }
}

// Check of the operator's values: out[0] = bits of max |a| over the finite
// entries, out[1] = bits of max |A(e, f) - A(f, e)^T| (the symmetry the method
// assumes: V = U in the compression), out[2] = number of non-finite entries.
// Non-negative doubles order like their bit patterns. grid: chunks over all entries.
template <class W>
__global__ __launch_bounds__(256) void validate_kernel(const W* __restrict__ vals, const int32_t* __restrict__ tblk,
                                                       int64_t nnzb, int q, unsigned long long* out) {
  const int64_t qq = (int64_t)q * q, tot = nnzb * qq;
  double amax = 0, dmax = 0;
  unsigned bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int64_t b = e / qq, rc = e % qq;
    const int c = (int)(rc / q), r = (int)(rc % q);
    const W v = vals[e];
    const W t = vals[(int64_t)tblk[b] * qq + (int64_t)r * q + c];  // entry (c, r) of block (f, e)
    const double a = sqrt((double)traits<W>::abs2(v));
    const double d = sqrt((double)traits<W>::abs2(v - t));
    if (!(a <= 1.7976931348623157e308) || !(d <= 1.7976931348623157e308)) {
      ++bad;
    } else {
      amax = fmax(amax, a);
      dmax = fmax(dmax, d);
    }
  }
  __shared__ double ra[256], rd[256];
  __shared__ unsigned rb[256];
  ra[threadIdx.x] = amax;
  rd[threadIdx.x] = dmax;
  rb[threadIdx.x] = bad;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      ra[threadIdx.x] = fmax(ra[threadIdx.x], ra[threadIdx.x + s]);
      rd[threadIdx.x] = fmax(rd[threadIdx.x], rd[threadIdx.x + s]);
      rb[threadIdx.x] += rb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(&out[0], (unsigned long long)__double_as_longlong(ra[0]));
    atomicMax(&out[1], (unsigned long long)__double_as_longlong(rd[0]));
    if (rb[0]) atomicAdd(&out[2], (unsigned long long)rb[0]);
  }
}

}  // namespace hss
