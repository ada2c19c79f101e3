/*
 * hss.h -- C ABI of the MI355X low-rank Schur-complement preconditioner.
 *
 * The library builds the approximate LDM^t factorization of a sparse matrix
 * given in element blocks (Gatto & Hesthaven, "A Preconditioner Based on
 * Low-Rank Approximation of Schur Complements", Section 3): nested
 * dissection over a binary tree of boxes, dense Schur complements at every
 * box, each compressed to HSS form by randomized interpolative
 * decompositions (Section 1, Theorem 1), merged level by level (equation
 * (32), Algorithm 2), and a dense root block (equation (36)). Its inverse
 * M^{-t} D^{-1} L^{-1} (end of Section 3.2) preconditions an FP64 GMRES.
 *
 * Conventions shared by every call:
 *   - Every call returns an hss_status_t; no C++ exception crosses the ABI.
 *     On a non-OK status hss_last_error() returns a message for the calling
 *     thread, output handles are set to NULL and nothing is leaked.
 *   - The caller owns every array it passes; the library copies what it
 *     keeps (the operator values, structure and tree).
 *   - Matrices and vectors are column-major. Complex scalars are
 *     interleaved (re, im) pairs of doubles (C99 double _Complex layout).
 *   - Device pointers belong to the device that is current when the handle
 *     is created; work is queued on opts.hip_stream (NULL = null stream).
 *   - One handle is used by one host thread / stream at a time.
 */
#ifndef HSS_H
#define HSS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hss_ctx* hss_handle_t;
typedef struct hss_plan_ctx* hss_plan_t;

typedef enum {
  HSS_OK = 0,
  HSS_EINVAL = -1,       /* bad argument, inconsistent structure or non-finite value */
  HSS_ENOMEM = -2,       /* host or device allocation failed                         */
  HSS_ESINGULAR = -3,    /* a pivot of some A^_ii (or of the root) is exactly zero    */
  HSS_ENOCONV = -4,      /* GMRES did not reach tol within maxit                      */
  HSS_EDEVICE = -5,      /* a HIP runtime call failed (no GPU, launch failure, ...)   */
  HSS_EUNSUPPORTED = -6  /* valid request outside what this library implements        */
} hss_status_t;

typedef enum { HSS_R64 = 0, HSS_C128 = 1 } hss_dtype_t;

/* Arithmetic of the factorization (Schur updates, compression, stored
 * factors). GMRES, the SpMV, the root block and all vectors stay FP64. */
typedef enum {
  HSS_PREC_FP64 = 0, /* everything in FP64 (complex128)                              */
  HSS_PREC_FP32 = 1, /* FP32 (complex64) factor, FP32 MFMA Schur products            */
  HSS_PREC_BF16 = 2  /* as FP32, but Schur products on BF16 MFMA with FP32 accumulate,
                        operands split in three BF16 terms (hi*hi + hi*lo + lo*hi);
                        real and complex operators                                     */
} hss_prec_t;

/* Element-block operator (Section 3.0: A is never assembled).
 * Block compressed rows over elements: block b of element row e couples the
 * q dofs of element e to the q dofs of element col_idx[b]; dof = elem*q + local.
 * vals holds nnzb blocks of q*q scalars, each column-major.
 * row_ptr / col_idx are host arrays; vals is host or device memory. */
typedef struct {
  int32_t n_el;
  int32_t q;
  const int32_t* row_ptr;  /* [n_el + 1]                    */
  const int32_t* col_idx;  /* [nnzb], ascending in each row  */
  const void* vals;        /* [nnzb * q * q] double or complex128 */
  hss_dtype_t dtype;
  int32_t vals_on_device;  /* 1: vals is a device pointer    */
} hss_block_op_t;

/* Separator tree (Algorithm 2 input: "binary tree partitioning the dofs").
 * Heap numbering: node 1 is the virtual root of the two top boxes 2 and 3
 * (the forest of Section 3.0), node s has children 2s and 2s+1. Only the
 * leaves are listed; inner boxes are unions of their leaves. Every inner
 * node must have both children. elem_xy gives integer grid coordinates of
 * each element; they fix the perimeter order of each box's boundary dofs. */
typedef struct {
  int32_t n_leaves;
  const int32_t* leaf_node;  /* [n_leaves] heap ids               */
  const int32_t* leaf_ptr;   /* [n_leaves + 1]                    */
  const int32_t* leaf_elems; /* [n_el] element ids, CSR by leaf    */
  const int32_t* elem_xy;    /* [2 * n_el] (x, y) per element      */
} hss_tree_t;

#define HSS_MLP_NPARAMS 4801 /* 8*64 + 64 + 64*64 + 64 + 64 + 1 */

typedef struct {
  hss_prec_t prec;
  int32_t p_os;            /* oversampling of the randomized ID (Theorem 1: 10) */
  int32_t l0;              /* initial sample count without a rank model (32)      */
  int32_t max_attempts;    /* judge / rank-growth rounds per box (8)              */
  uint64_t seed;           /* Philox key of the Gaussian test matrices            */
  const float* rank_model; /* NULL: plain adaptive ID; else HSS_MLP_NPARAMS host
                              floats (W1,b1,W2,b2,W3,b3, row-major [out][in]) of
                              the rank predictor that presizes l per box as
                              32 * ceil((m k^ + p_os) / 32), k^ its prediction and
                              m = model_margin                                    */
  double kappa_h;          /* wavenumber * element size, a rank-model feature    */
  void* hip_stream;        /* hipStream_t for all work (NULL: null stream)       */
  int32_t profile;         /* 0: off; 1: time every kernel class with HIP events on
                              hip_stream; otherwise bit (c + 1) times class c in the
                              order of the hss_query "prof." classes            */
  int32_t apply_graph;     /* 1 (default): the apply sweeps run as a captured HIP
                              graph, one per right-hand-side count; 0: eager      */
  int32_t hss_leaf_elems;  /* leaves of the HSS tree over a box's boundary: at most
                              this many elements (0: the default, 4)               */
  const char* rank_model_path; /* weights file written by hss_rank_model_train, read
                              when rank_model is NULL (NULL: no file)            */
  int32_t keep_box;        /* heap id of one box of problem 0 whose Schur complement
                              S (symmetrized, before compression) and compressed S~
                              the handle keeps for hss_query "kept_S" / "kept_St"
                              (0: none; HSS_EINVAL if no such box)                */
  int32_t ldu;             /* storage of the eliminated interiors of more than 128
                              rows and of the root: 0 explicit inverses, 1 block LDU
                              form (a third of the inverse's work, two GEMV launches
                              per block in each apply), 2 (default) the LDU form for
                              the batches where the work saved outweighs the added
                              launches                                            */
  double model_margin;     /* samples per predicted rank, m above (0: the default,
                              3; otherwise at least 1)                            */
} hss_opts_t;

typedef struct {
  int32_t iters;       /* Arnoldi steps (matvecs with A M^{-1})  */
  int32_t restarts;
  double true_relres;  /* ||b - A x|| / ||b|| in FP64 at exit     */
  int32_t status;      /* HSS_OK or HSS_ENOCONV                  */
} hss_gmres_info_t;

/* Fill *o with the defaults (FP32, p_os 10, l0 32, 8 attempts, seed 1508, HSS
 * leaves of 4 elements). */
void hss_default_opts(hss_opts_t* o);

/* hss_factor -- build the preconditioner of one operator (Algorithm 2 plus
 * the root of equation (36)).
 *   A, T   operator and tree as above (validated; HSS_EINVAL on any
 *          inconsistency, HSS_EUNSUPPORTED for a structurally nonsymmetric A).
 *   tol    relative Frobenius tolerance of every box's HSS compression,
 *          ||S - S~||_F <= tol ||S||_F (the norm Section 1 leaves open);
 *          tol = 0 skips compression and gives the exact factorization.
 *   o      options (NULL: defaults).
 *   out    receives the handle; free with hss_destroy.
 * Returns HSS_ESINGULAR if a pivot is exactly zero (hss_last_error names the box). */
hss_status_t hss_factor(const hss_block_op_t* A, const hss_tree_t* T, double tol,
                        const hss_opts_t* o, hss_handle_t* out);

/* hss_factor_batched -- nprob independent operators factorized together,
 * one launch per kernel per height wave across all problems (the boxes of one
 * level are independent, Section 3). The handle's vectors are the
 * concatenation of the problems' dofs, problem 0 first. */
hss_status_t hss_factor_batched(int32_t nprob, const hss_block_op_t* A, const hss_tree_t* T,
                                double tol, const hss_opts_t* o, hss_handle_t* out);

/* hss_apply -- y = M^{-t} D^{-1} L^{-1} x (end of Section 3.2) for nrhs
 * columns. x, y: arrays of FP64 (complex128 for complex operators), leading
 * dimensions ldx, ldy >= total dofs, in the caller's dof order; x and y may not
 * overlap. on_device = 1: device arrays (work queued on the handle's stream,
 * returns after it); 0: host arrays (copied to the device and back). */
hss_status_t hss_apply(hss_handle_t h, int32_t nrhs, const void* x, int64_t ldx, void* y,
                       int64_t ldy, int32_t on_device);

/* gmres_solve -- right-preconditioned restarted GMRES(restart) in FP64 on the
 * device for every (problem, column) system. b, x: arrays [ld x nrhs], device
 * arrays if on_device = 1, host arrays (copied both ways) if 0; x holds the
 * initial guess on entry and the solution on exit (x = 0 for a zero b). info:
 * host array [nprob * nrhs] (problem-major). Stops a system when its rotated
 * residual and then its true residual are <= tol. Returns HSS_ENOCONV if any
 * system missed tol within maxit Arnoldi steps (x holds the last iterate). */
hss_status_t gmres_solve(hss_handle_t h, int32_t nrhs, const void* b, void* x, int64_t ld,
                         double tol, int32_t restart, int32_t maxit, int32_t on_device,
                         hss_gmres_info_t* info);

/* hss_query -- read a diagnostic of the handle into out[0..cap).
 * *len receives the number of values the key has (also when cap is smaller).
 * Keys: "n" (total dofs), "nprob", "nnodes", "nwaves", "max_err", "ranks"
 * (largest ID rank per box), "attempts" (per box), "l" (final sample count per
 * box), "l_init" (first sample count per box: l0, or the rank model's size), "err" (per box judge error), "node_heap" / "node_prob" / "node_ni" /
 * "node_nb" (per box), "features" (8 per box), "tmax" (per box, largest
 * |interpolation coefficient|), "fallbacks", "retries",
 * "flops_factor" (the method's work by formula, real flops, complex x4: LU
 * (2/3) n_i^3 + triangular solves 2 n_i^2 n_b + Schur product 2 n_b^2 n_i per box,
 * the root's LU, and the sampling and truncated QR of every compression attempt
 * from the ranks chosen), "flops_factor_parts" (those six terms), "flops_gj" (the
 * work of the elimination the library executes: Gauss-Jordan inverses of the
 * interiors of at most 128 rows, the block LDU form of the larger ones and of the
 * root, and the Schur products),
 * "bytes_apply", "bytes_spmv", "time_factor_ms", "host_wait_ms"
 * (time the factorization spent waiting for the device at its sync points),
 * "root_block" (block width of the roots' block LDU form; 0: explicit inverses),
 * "cpqr_queue_launches" (truncated-QR launches that ran as a persistent work
 * queue: HSS heights of more nodes than the device holds at once, when the
 * environment sets HSS_CPQR_QUEUE=1; 0 otherwise),
 * "compress_host_ms" (4 values: host time of the compression attempts spent
 * building and uploading their lists, launching, waiting for the judge, and
 * deciding the next attempt),
 * "phase_ms" (8 values: host wall time of operator upload, features and the
 * rank model's inference (one device launch for all boxes), gather,
 * Gauss-Jordan, Schur GEMM, compression, root, apply set-up),
 * "prof.<class>.ms|launches|flops|bytes" (HIP-event time, launch count and
 * algorithmic work of the timed launches) for the classes, in bit order:
 * gather, gj_panel, gj_rows, gj_update, gj_perm, schur_gemm, symm, omega,
 * sample_gemm, sample, id, utall, expand, judge, root, apply, spmv, gmres. */
hss_status_t hss_query(hss_handle_t h, const char* key, double* out, int64_t cap, int64_t* len);

void hss_destroy(hss_handle_t h);

/* Message of the calling thread's last non-OK status (empty if none). */
const char* hss_last_error(void);

/* ---- host-only planning (no GPU needed) --------------------------------
 * hss_plan_create runs the planner of hss_factor (boundary / interior sets,
 * orderings, height waves, HSS trees with leaves of at most hss_leaf_elems
 * elements, 0 for the default 4) on the host and keeps the result for
 * inspection. hss_plan_query keys, per box `node` (heap id):
 *   "idof" / "bdof"  I^ (interior) and B (boundary) dofs in factor order,
 *   "hss"            HSS tree as (lo, hi, left, right) quadruples, post-order,
 *                    left/right = -1 for leaves,
 *   "height"         wave index;
 * and with node = 1: "root" (the dofs of the root block). Values are int64. */
hss_status_t hss_plan_create(const hss_block_op_t* A, const hss_tree_t* T, int32_t hss_leaf_elems,
                             hss_plan_t* out);
hss_status_t hss_plan_query(hss_plan_t p, const char* key, int32_t node, int64_t* out,
                            int64_t cap, int64_t* len);
void hss_plan_destroy(hss_plan_t p);

/* Tuning table of the Gauss-Jordan kernels that eliminate the box interiors, as
 * written by the project's autotuner (paper_1508_07798_amd/autotune.py): per
 * scalar type (0 float, 1 double, 2 complex float, 3 complex double) and size
 * class (boxes of at most 128, 256, 512, 1024, 2048 or 4096 interior rows) a
 * compact panel shape (width nb, rows per thread rpt, threads nt; nt = 0 keeps
 * the built-in choice) and a second-level block width (-1: built-in, 0: none,
 * else at most 256 columns). The library reads tuning_gfx950.json beside
 * libhss.so at the first factorization ($HSS_TUNING names another file; an empty
 * value: none) unless a call below has set the table first. An entry whose shape is not compiled or holds fewer rows than a
 * box is ignored for that box. The table is process-wide; changing it while
 * another thread factorizes is a race.
 *   hss_tuning_load        reads a JSON file {"entries": [{"scalar": "complex64",
 *                          "rows": 1024, "nb": 16, "rpt": 4, "nt": 256,
 *                          "block": 128}, ...]}; HSS_EINVAL if malformed
 *   hss_tuning_set         one entry (rows_class one of the class sizes)
 *   hss_tuning_clear       back to the built-in rules
 *   hss_tuning_candidates  the compiled shapes that hold `rows` rows: (nb, rpt, nt)
 *                          triples into out (host, at most cap), *count all of them */
hss_status_t hss_tuning_load(const char* path);
hss_status_t hss_tuning_set(int32_t scalar, int32_t rows_class, int32_t nb, int32_t rpt, int32_t nt,
                            int32_t block);
void hss_tuning_clear(void);
hss_status_t hss_tuning_candidates(int32_t scalar, int32_t rows, int32_t* out, int32_t cap, int32_t* count);

/* ---- rank-predictor MLP (8 -> 64 -> 64 -> 1, tanh) ---------------------
 * Not in the paper: it replaces the anticipated rank of Section 4 by a
 * learned prediction. Device pointers; weights as in hss_opts_t.rank_model.
 * hss_mlp_forward: y[n] = f(x[n x 8] row-major).
 * hss_mlp_grad: grad[HSS_MLP_NPARAMS] and *loss of the mean squared error
 *   against target[n] (host *loss).
 * hss_mlp_train: `steps` full-batch Adam steps (beta 0.9 / 0.999, eps 1e-8)
 *   updating weights in place; loss_hist[steps] (device) gets each loss. */
hss_status_t hss_mlp_forward(const float* weights, const float* x, int32_t n, float* y,
                             void* hip_stream);
hss_status_t hss_mlp_grad(const float* weights, const float* x, const float* target, int32_t n,
                          float* grad, double* loss, void* hip_stream);
hss_status_t hss_mlp_train(float* weights, const float* x, const float* target, int32_t n,
                           int32_t steps, float lr, float* loss_hist, void* hip_stream);

/* hss_rank_model_train -- train the rank predictor on (features, rank) samples
 * and write its weights to out_path, a file that hss_opts_t.rank_model_path can
 * name. feat: host [n x 8] row-major (the "features" of hss_query), rank: host
 * [n] (the "ranks" of the same boxes). Weights start N(0, 1/fan_in) from a
 * stream keyed by seed; 1500 full-batch Adam steps on the device (learning rate
 * 3e-3) fit log2(1 + rank). HSS_EINVAL for non-finite inputs or an unwritable
 * path. File layout: "HSSMLP01", int32 count, count float32 (little-endian). */
hss_status_t hss_rank_model_train(const float* feat, const float* rank, int32_t n, const char* out_path,
                                  uint64_t seed);

/* hss_mlp_grad_noalloc -- hss_mlp_grad without any device allocation, for
 * callers that cannot allocate (code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid hipMalloc). The gradient pass keeps its
 * activations and partial terms in a fixed device array of the library
 * (HSS_MLP_NOALLOC_MAX_N samples, about 8.5 MB, held on every device the library
 * runs on until the process ends); grad and loss are as in hss_mlp_grad.
 * Returns HSS_EINVAL for n < 1 or n > HSS_MLP_NOALLOC_MAX_N. Every call on one
 * device uses the same array, so calls that overlap on one device (other
 * streams, other threads) race; serialize them. */
#define HSS_MLP_NOALLOC_MAX_N 8192
hss_status_t hss_mlp_grad_noalloc(const float* weights, const float* x, const float* target, int32_t n,
                                  float* grad, double* loss, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* HSS_H */
