/*
 * hss_debug.h -- kernel-level entry points of libhss used by the test suite
 * to check single building blocks of the factorization on the device.
 * Same conventions as hss.h (status codes, hss_last_error, column-major,
 * device pointers, work on `hip_stream`, returns after the stream is synced).
 *
 * scalar codes: 0 = float, 1 = double, 2 = complex float, 3 = complex double;
 * hss_debug_gemm also takes 4 = float operands on BF16 matrix cores (each value
 * split into bf16 hi + lo parts, three products, FP32 accumulation: the Schur
 * update of the HSS_PREC_BF16 factorization), 5 = complex float operands on
 * BF16 matrix cores (the same split for each of the four real products), and
 * 6 = float on the 128 x 128-tile MFMA kernel that the factorization uses for its
 * large real FP32 products.
 */
#ifndef HSS_DEBUG_H
#define HSS_DEBUG_H

#include <stdint.h>

#include "hss.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C_b = alpha A_b B_b + beta C_b for b < nbatch (the batched MFMA GEMM of the
 * Schur updates, equation (32)). Arrays of device pointers and sizes are host
 * arrays; alpha, beta are (re, im) pairs. */
hss_status_t hss_debug_gemm(int32_t scalar, int32_t nbatch, const void* const* A, const void* const* B,
                            void* const* C, const int32_t* M, const int32_t* N, const int32_t* K,
                            const int32_t* lda, const int32_t* ldb, const int32_t* ldc,
                            const double* alpha, const double* beta, void* hip_stream);

/* In-place [A_b | B_b] -> [A_b^{-1} | A_b^{-1} B_b] (n_b x (n_b + m_b), ld n_b) by
 * the blocked Gauss-Jordan elimination with partial pivoting that the
 * factorization uses for every A^_ii. block = 0 keeps the factorization's own
 * choice of second-level blocking; block in [1, 256] forces blocks of that many
 * pivot columns (HSS_EINVAL outside [0, 256]). Complex64 batches whose largest
 * box has more than 2048 rows run their panels in complex128 on a widened copy of
 * each block (the block products stay complex64), as the factorization does.
 * *singular receives 1 if a pivot was 0. */
hss_status_t hss_debug_gj(int32_t scalar, int32_t nbatch, void* const* Mat, const int32_t* n,
                          const int32_t* m, int32_t block, int32_t* singular, void* hip_stream);

/* Row interpolative decomposition of one candidate set (Section 1: the ID with
 * interpolation coefficients bounded by 2 in modulus), as the compression runs it
 * on every HSS node: column-pivoted Householder QR of Z^T truncated at the first k
 * with ||R22||_F <= thresh, then strong-RRQR swaps while max |T| > 2.
 *   Zt     device, l x m column-major: Z^T for the m candidate rows of Z (m x l),
 *          i.e. Z in row-major order; not modified. 1 <= m <= 1024, 1 <= l <= 512.
 *   p_os   oversampling used for the "samples exhausted" test (k + p_os > l).
 *   k      host: the rank.   skel  host [m]: the first k entries are the skeleton
 *          rows in skeleton order.   U  device, m x min(l, m) column-major (ld m):
 *          Z ~= U(:, 0:k) Z(skel, :); U(skel(i), i) = 1.
 *   tmax   host: max |T| after the swaps. */
hss_status_t hss_debug_row_id(int32_t scalar, const void* Zt, int32_t m, int32_t l, double thresh, int32_t p_os,
                              int32_t* k, int32_t* skel, void* U, float* tmax, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* HSS_DEBUG_H */
