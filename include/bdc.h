/*
 * bdc.h -- C ABI of the MI355X bidiagonal divide-and-conquer SVD.
 *
 * Computes B = U diag(sigma) V^T for an n x n real upper bidiagonal B with
 * diagonal d (length n) and superdiagonal e (length n-1), with full singular
 * vectors, in IEEE binary64.  This is the bidiagonal SVD stage of the paper's
 * GPU-centered SVD (Section 4.2, "Diagonalization"; the BDC algorithm of
 * Algorithm 2 with the deflation of Algorithm 3 and the merge of Algorithm 4).
 * The result satisfies sigma_1 >= ... >= sigma_n >= 0 with U and V orthogonal
 * (the SVD definition of Section 1).
 *
 * Memory.  Every matrix and vector argument is a device pointer on the device
 * the handle was created for.  Matrices are column-major with leading
 * dimension n.  The caller owns all arguments; inputs are never written;
 * outputs are overwritten entirely and are also used as scratch during the
 * call.  The handle owns its workspace (grown on demand, kept between calls).
 *
 * Streams.  Every compute call only enqueues work on `stream` and returns;
 * nothing synchronises the device.  A handle may be used by one host thread
 * at a time, and calls on one handle must not overlap on different streams.
 *
 * Errors.  Every function returns a status: BDC_OK (0); -i when argument i
 * (1-based) is invalid, detected on the host before any device work; or one
 * of the negative BDC_ERR_* codes below.  Conditions found on the device
 * (non-finite input, iteration caps) are reported by bdc_get_info after the
 * stream has been synchronised.
 */
#ifndef BDC_H_
#define BDC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bdc_handle_s* bdc_handle_t;
typedef void* bdc_stream_t; /* a hipStream_t; NULL = the default stream */

enum {
  BDC_OK = 0,
  BDC_ERR_INVALID_HANDLE = -1001, /* NULL or destroyed handle */
  BDC_ERR_NO_DEVICE = -1002,      /* no HIP device, or device index out of range */
  BDC_ERR_NOMEM = -1003,          /* workspace would exceed the cap, or hipMalloc failed */
  BDC_ERR_HIP = -1004,            /* a HIP runtime call failed */
  BDC_ERR_NONFINITE = -1005,      /* (info) d or e holds Inf or NaN */
  BDC_ERR_UNSUPPORTED = -1006,    /* option value not supported by this library */
  BDC_ERR_NO_MODEL = -1007,       /* learned start requested before bdc_mlp_set */
  BDC_ERR_TOO_LARGE = -1008       /* beyond the fixed scratch of an allocation-free entry point */
};

/* Start of the secular iteration (options.start). */
enum {
  BDC_START_PLAIN = 0,  /* first evaluation at the interval's midpoint in omega^2 */
  BDC_START_LEARNED = 1 /* first evaluation at the position proposed by the MLP */
};

/* Arithmetic of the vector-update products (options.gemm). */
enum {
  BDC_GEMM_FP64 = 0, /* FP64 matrix cores (the paper's FP64 products) */
  BDC_GEMM_OZAKI = 1, /* split precision: bfloat16 digit slices on the bfloat16 matrix
                         cores, FP32 accumulation, FP64 combination (single-problem
                         solves; batched solves keep FP64) */
  BDC_GEMM_CRT = 2    /* split precision: the integer product of the power-of-two
                         scaled operands formed exactly from int8 residues modulo
                         crt_moduli coprime moduli on the int8 matrix cores (int32
                         accumulation) and rebuilt by the Chinese remainder theorem
                         (single-problem solves; batched solves keep FP64) */
};

/* Size of the learned-start network: 19 features -> 64 -> 64 -> 64 -> 1. */
#define BDC_MLP_FEATURES 19
#define BDC_MLP_HIDDEN 64
#define BDC_MLP_PARAMS (19 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 + 1)

/* Options; bdc_default_options fills the defaults. */
typedef struct {
  int leaf_size;              /* largest leaf (rows), 4..32; default 32 (Section 4.2.2: 32 was best) */
  int max_secular_iters;      /* evaluations of the secular function per root, 2..64; default 64 */
  int max_leaf_sweeps;        /* QR sweeps per leaf row, 1..1000; default 40 (cap = value * m) */
  size_t workspace_cap_bytes; /* 0 = unlimited */
  int timing;                 /* 1: record per-kernel event times (bdc_get_timing); launches
                                 kernels one by one (no graph) */
  int use_graph;              /* 1 (default): capture a solve's launch sequence once per
                                 (sizes, buffers) as a HIP graph and replay it */
  int start;                  /* BDC_START_PLAIN (default) or BDC_START_LEARNED (needs
                                 bdc_mlp_set first; same stopping rule, only the
                                 first point of each root's iteration changes) */
  int gemm;                   /* BDC_GEMM_FP64 (default) or BDC_GEMM_OZAKI */
  int ozaki_slices;           /* slices per operand, 5..7 (default 7: terms dropped
                                 below about 2^-54 relative to |row| |column|; 6
                                 leaves about 2^-46, which at n = 16384 exceeds a
                                 1e-12 residual) */
  int ozaki_min_n;            /* merges with at least this many kept values use the
                                 split products (either form), >= 128 (default 256);
                                 smaller ones FP64 */
  int crt_moduli;             /* moduli of BDC_GEMM_CRT, 13..16 (default 16: operands
                                 rounded at 2^-54 of each row's / column's largest
                                 entry for products up to 16384 deep) */
  int learned_min_n;          /* with BDC_START_LEARNED, the network proposes the
                                 first points of merges of at least this many kept
                                 values only; smaller merges start at the midpoint,
                                 where one evaluation costs less than the network
                                 (default BDC_LEARNED_MIN_N; 0 = every merge) */
} bdc_options_t;
#define BDC_LEARNED_MIN_N 1024

void bdc_default_options(bdc_options_t* opt);

/* Create a handle on HIP device `device`.  opt may be NULL (defaults).
 * Returns BDC_ERR_NO_DEVICE when the device does not exist. */
int bdc_create(bdc_handle_t* handle, int device, const bdc_options_t* opt);

/* Wait for the handle's outstanding work, then free it and its workspace. */
int bdc_destroy(bdc_handle_t handle);

/* B = U diag(sigma) VT for one n x n upper bidiagonal (Algorithm 2).
 *   n      >= 0 (0 is a no-op)
 *   d      device, n doubles (diagonal)
 *   e      device, n-1 doubles (superdiagonal); may be NULL when n <= 1
 *   sigma  device, n doubles, out: descending, >= 0
 *   U      device, n*n doubles, column-major, out: left singular vectors
 *   VT     device, n*n doubles, column-major, out: V^T (row i = right vector i)
 *   stream the HIP stream to enqueue on
 * U and VT must not overlap each other or the inputs. */
int bdc_svd(bdc_handle_t handle, int64_t n, const double* d, const double* e,
            double* sigma, double* U, double* VT, bdc_stream_t stream);

/* Many independent bidiagonals of uneven sizes in one call; merge levels of
 * all problems run together (the independent subproblems noted in Section
 * 4.2.2).
 *   batch   >= 0 problems; sizes  host array of `batch` sizes n_i >= 0
 *   d, e    device, packed: problem i at offset off_i = sum_{j<i} n_j (e uses
 *           the same offsets; its entry off_i + n_i - 1 is ignored)
 *   sigma   device, packed like d
 *   U, VT   device, packed: problem i at offset sum_{j<i} n_j^2, each
 *           n_i x n_i column-major */
int bdc_svd_batched(bdc_handle_t handle, int64_t batch, const int64_t* sizes,
                    const double* d, const double* e, double* sigma, double* U,
                    double* VT, bdc_stream_t stream);

/* Diagnostics of the last bdc_svd / bdc_svd_batched call; valid once its
 * stream has been synchronised (this call synchronises the handle's stream).
 *   info  out (may be NULL): 0 on success, BDC_ERR_NONFINITE when the input
 *         held Inf/NaN, else the number of leaves plus secular roots that hit
 *         their iteration cap (their results are the last iterate).
 *   stats out (may be NULL): counters, see bdc_stats_t. */
typedef struct {
  int64_t merges;              /* merge nodes solved */
  int64_t roots;               /* secular roots solved (sum of N over merges) */
  int64_t secular_evals;       /* evaluations of the secular function (sum over roots) */
  int64_t deflated_small_z;    /* deflations by small z component */
  int64_t deflated_zero_d;     /* deflations of values within tol of 0 */
  int64_t deflated_close;      /* deflations of close value pairs */
  int64_t rotations;           /* Givens rotations applied by deflation */
  double update_flops;         /* flops of the vector-update products actually executed */
  int64_t root_N;              /* non-deflated size at the root merge (first problem) */
  int64_t levels;              /* merge levels */
  int64_t secular_terms;       /* pole terms summed by the secular evaluations */
  double leaf_flops;           /* flops of the rotations applied by the leaf solves */
  double gather_bytes;         /* bytes moved gathering the kept columns (read + write) */
  int64_t final_read_elems;    /* nonzero-support entries read to write U and V^T */
  int64_t split_merges;        /* merges whose update products took the split form */
  double split_flops;          /* their share of update_flops */
} bdc_stats_t;

int bdc_get_info(bdc_handle_t handle, int64_t* info, bdc_stats_t* stats);

/* Per-kernel times, when options.timing = 1, summed over the calls since the
 * handle was created or bdc_clear_timing was last called.  Each launch is
 * bracketed by HIP events on the call's stream.  Synchronises the stream,
 * fills up to `cap` entries of kernel names / total milliseconds / launch
 * counts and returns the number of kernel kinds. */
int bdc_get_timing(bdc_handle_t handle, int cap, const char** names, double* ms,
                   int64_t* launches);
int bdc_clear_timing(bdc_handle_t handle);

/* ---- single-step entry points ------------------------------------------
 * They run one stage of a merge through the same device code as bdc_svd, on
 * caller-provided inputs, so each stage can be compared with an independent
 * implementation on identical inputs.  All arrays are device pointers. */

/* Leaf SVD by QR iteration (Algorithm 2 step (1)) of the m x (m+s) upper
 * bidiagonal with diagonal d (m) and superdiagonal e (m-1+s; with s = 1 the
 * last entry is in column m+1).  1 <= m <= 32, s in {0,1}.
 * Out: sigma (m, ascending), W (m*m, col-major), Q ((m+s)^2, col-major, the
 * last column spans the null space when s = 1). */
int bdc_step_leaf(bdc_handle_t handle, int m, int s, const double* d, const double* e,
                  double* sigma, double* W, double* Q, bdc_stream_t stream);

/* z formation, sort and deflation of one merge (Algorithm 3).
 *   m, s, k = m/2: node size; sig  (m) children's values (sig[0..k-2] the
 *   left child's, ascending; sig[k-1] ignored; sig[k..m-1] the right child's,
 *   ascending); qrow1 (k): last row of the left child's right basis, qrow1[k-1]
 *   = last entry of its null vector; qrow2 (m-k+s): first row of the right
 *   child's right basis, qrow2[m-k] = first entry of its null vector if s=1;
 *   alpha, beta: the middle row's entries (Section 4.2.1 divide step).
 * Out (device):
 *   perm   (m int32): sorted position -> node column (middle = k-1 first)
 *   dz     (2m doubles): values then z at sorted positions after deflation,
 *          scaled by the power of two `scale`
 *   status (m int32): 0 kept, 1 small z, 2 value within tol of 0, 3 close pair
 *   rot_pos (2m int32) and rot_cs (2m doubles): rotation r rotates sorted
 *          positions (rot_pos[2r], rot_pos[2r+1]) with (c, s) =
 *          (rot_cs[2r], rot_cs[2r+1]); kind 2 when rot_pos[2r] = 0, else 3
 *   misc   (8 doubles): scale, tol, c0, s0, N, n1, n2, n3 (counts as doubles)
 *   nrot   (1 int32): number of rotations. */
int bdc_step_deflate(bdc_handle_t handle, int m, int s, const double* sig,
                     const double* qrow1, const double* qrow2, double alpha, double beta,
                     int32_t* perm, double* dz, int32_t* status, int32_t* rot_pos,
                     double* rot_cs, double* misc, int32_t* nrot, bdc_stream_t stream);

/* Roots of the secular equation 1 + sum_j z_j^2/(d_j^2 - w^2) = 0 (eq.
 * M-svd-val) for d (N, strictly increasing, d[0] = 0) and z (N, no zero):
 * w_i = d[o_i] + tau_i; iters = evaluations per root. */
int bdc_step_secular(bdc_handle_t handle, int N, const double* d, const double* z,
                     int32_t* o, double* tau, int32_t* iters, bdc_stream_t stream);

/* As bdc_step_secular, with each root's iteration started from a proposed
 * position xstart[i] in (0, 1) of its interval (device, N floats; NULL = the
 * plain midpoint start).  Interval of root i: (d_i, d_{i+1}), the last root's
 * (d_{N-1}, sqrt(d_{N-1}^2 + sum z^2)). */
int bdc_step_secular_start(bdc_handle_t handle, int N, const double* d, const double* z,
                           const float* xstart, int32_t* o, double* tau, int32_t* iters,
                           bdc_stream_t stream);

/* Features of the learned start for the secular problem (d, z) as above:
 * X (device, N x BDC_MLP_FEATURES floats, row-major).  Feature layout: for the
 * 4 poles at and below root i and the 4 above it, the gap (d_j - lo)/h and
 * the strength log2(z_j^2/(hi^2 - lo^2))/32; then log2(rho/(hi^2 - lo^2))/32
 * and the far field (the secular function without those 8 poles, summed
 * term by term in nearby blocks and by one monopole per distant block) at
 * the interval's midpoint: asinh(value)/8, asinh(slope (hi^2 - lo^2))/8. */
int bdc_step_features(bdc_handle_t handle, int N, const double* d, const double* z, float* X,
                      bdc_stream_t stream);

/* Recomputed z (eq. bdc-zi) and the normalised singular vectors of
 * M~ = e_1 zt^T + diag(d) (eq. M-svd-vec), from d, z, o, tau as above.
 * Out: zt (N), UM and VM (N*N col-major, column i belongs to root i). */
int bdc_step_vectors(bdc_handle_t handle, int N, const double* d, const double* z,
                     const int32_t* o, const double* tau, double* zt, double* UM,
                     double* VM, bdc_stream_t stream);

/* C (M x N, ldc) = A (M x K, lda) * B (K x N, ldb), column-major, with the
 * FP64 matrix-core kernel of the vector update (eq. bdc-Mv2Bv-u-vt). */
int bdc_step_gemm(bdc_handle_t handle, int M, int N, int K, const double* A, int lda,
                  const double* B, int ldb, double* C, int ldc, bdc_stream_t stream);

/* ---- back-transformation of singular vectors -------------------------------
 * The step after the bidiagonal SVD on the paper's full-SVD path (Section
 * 4.3.3): U = U_1 U_2 and V^T = V_2^T V_1^T, where U_1 = H_0 ... H_{n-1} and
 * V_1 = G_0 ... G_{n-2} are the products of the column and row Householder
 * reflectors of the bidiagonal reduction (Section 4.1) and U_2, V_2 the
 * bidiagonal's singular vectors (bdc_svd).  Both are C <- Q C with Q a
 * product of reflectors: U = Q_col [U_2; 0], and V = P_row V_2 (then V^T).
 *
 * C (m x p, column-major, ld ldc >= m) <- Q C (trans = 0) or Q^T C
 * (trans = 1), Q = H_0 H_1 ... H_{k-1}, H_i = I - tau[i] y_i y_i^T.  y_i has
 * a unit pivot at row i + offset, zeros above it, and below it the entries
 * Y[r * y_rs + i * y_cs] (LAPACK's geqrf / gebrd storage: column-stored
 * reflectors y_rs = 1, y_cs = ld; row-stored ones y_rs = ld, y_cs = 1, with
 * offset 1 for gebrd's row reflectors); tau[i] = 0 makes H_i the identity.
 * All pointers are device pointers; Y and tau are not written.  The
 * reflectors are applied `block` at a time (1..64; 0 = 64) in the modified
 * compact WY form of eq. inv_t / larft_update: T^{-1} = Y^T Y above its
 * diagonal and 1/tau_i on it (gemm), Z = Y^T C (gemm), Z = T^{-1} \ Z (trsm),
 * C = C - Y Z (gemm), on the FP64 matrix cores.  Scratch is owned by the
 * handle (grown on demand).  Enqueues on `stream`; returns BDC_OK, -i for an
 * invalid argument i, BDC_ERR_NOMEM or BDC_ERR_HIP. */
int bdc_apply_reflectors(bdc_handle_t handle, int trans, int m, int p, int k, int offset, const double* Y,
                         int64_t y_rs, int64_t y_cs, const double* tau, double* C, int ldc, int block,
                         bdc_stream_t stream);

/* bdc_apply_reflectors for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results (bit for bit), but the
 * scratch is a fixed 32 MiB array of device memory per GPU, held until the
 * process ends, and C is transformed in panels of at most 512 columns.  No
 * hipMalloc, hipFree or allocating library call is made.  Limit:
 * 8 (m b + b^2 + 33 b max(b, min(p, 512))) + 1024 <= 32 MiB for the block
 * size b (m <= 48574 with b = 64 and p >= 512, any k); larger problems return
 * BDC_ERR_TOO_LARGE before any work is enqueued.  Every call on one GPU shares
 * that GPU's array (which keeps the last call's contents; nothing in it needs
 * to start at zero): calls that overlap in time on one GPU, from any handle
 * or stream, race and must be ordered by the caller.  Returns as
 * bdc_apply_reflectors, or BDC_ERR_TOO_LARGE, or BDC_ERR_HIP when the
 * array's address could not be found when the handle was created. */
int bdc_apply_reflectors_noalloc(bdc_handle_t handle, int trans, int m, int p, int k, int offset,
                                 const double* Y, int64_t y_rs, int64_t y_cs, const double* tau, double* C,
                                 int ldc, int block, bdc_stream_t stream);

/* ---- bidiagonal reduction -----------------------------------------------------
 * The step before the bidiagonal SVD on the paper's dense path (Section 4.1,
 * Algorithm 1, the merged-rank-(2b) gebrd): B = Q^T A P with Q = H_0 ...
 * H_{n-1}, P = G_0 ... G_{n-2}.
 *
 * bdc_gebrd: A (m x n, column-major, ld lda >= m, m >= n, device) is
 * overwritten in LAPACK's gebrd storage: d on the diagonal, e on the
 * superdiagonal, the column reflectors below the diagonal (H_i: unit pivot
 * at row i) and the row reflectors right of the superdiagonal (G_i: unit
 * pivot at column i + 1); d (n), e (n - 1), tauq (n), taup (n, taup[n-1] =
 * 0) are device outputs.  Panels of `block` columns and rows (1..32; 0 = 32)
 * are reduced by one cooperative grid each (eq. bidiag-y-k3, bidiag-x-k3:
 * two passes over the panel-start trailing matrix per column, five grid
 * barriers per column), then the trailing matrix is updated by the one
 * product A - P Q^T (eq. bidiag-A-trail3) on the FP64 matrix cores.  With
 * bdc_svd(d, e) = U_2 Sigma V_2^T it gives the dense SVD: U = Q [U_2; 0] by
 * bdc_apply_reflectors on the column reflectors (y_rs = 1, y_cs = lda,
 * offset 0, tauq) and V = P V_2 on the row reflectors (y_rs = lda, y_cs = 1,
 * offset 1, taup).  Returns BDC_OK, -i for argument i, BDC_ERR_NOMEM or
 * BDC_ERR_HIP. */
int bdc_gebrd(bdc_handle_t handle, int m, int n, double* A, int lda, double* d, double* e, double* tauq,
              double* taup, int block, bdc_stream_t stream);

/* ---- tall-and-skinny QR ---------------------------------------------------
 * The first step of the paper's SVD of a tall matrix (Section 4.3.1-4.3.2):
 * A = Q R, then the SVD of the small R, and U = Q [U_0; 0].
 *
 * bdc_geqrf: A (m x n, column-major, ld lda >= m, m >= n, device) is
 * overwritten with R on and above the diagonal and the Householder vectors
 * below it, tau (n, device) with their scalars -- LAPACK's geqrf storage,
 * H_i = I - tau_i y_i y_i^T with y_i = 1 at row i.  Blocked: panels of
 * `block` columns (1..64; 0 = 32) are factored on the GPU one column at a
 * time by a cooperative grid (one grid all-reduce per column), and the
 * trailing columns are updated by the panel's reflectors in the modified
 * compact WY form of eq. inv_t / larft_update (T^{-1} = Y^T Y, gemm, trsm,
 * gemm).  The rows below a panel's top block must fit the resident grid (at
 * most 10240 / block rows per workgroup, one workgroup per CU: m - j0 - block
 * <= 40960 at block 64 and 81920 at block 32 on a 256-CU device), else
 * BDC_ERR_TOO_LARGE.  Returns BDC_OK, -i for argument i, BDC_ERR_NOMEM,
 * BDC_ERR_TOO_LARGE or BDC_ERR_HIP. */
int bdc_geqrf(bdc_handle_t handle, int m, int n, double* A, int lda, double* tau, int block,
              bdc_stream_t stream);

/* bdc_orgqr: Q (m x ncols, column-major, ld ldq >= m, device) <- the first
 * ncols columns of H_0 H_1 ... H_{k-1} (k <= ncols <= m; reflectors as
 * bdc_geqrf leaves them in A, ld lda), eq. orgqr-q: the identity multiplied
 * by the blocks of `block` reflectors (1..64; 0 = 64) from the last to the
 * first, T^{-1} of each block computed afresh (its own block size, not
 * geqrf's), block j touching only the rows and columns from its first pivot
 * on.  Returns BDC_OK, -i for argument i, BDC_ERR_NOMEM or BDC_ERR_HIP. */
int bdc_orgqr(bdc_handle_t handle, int m, int ncols, int k, const double* A, int lda, const double* tau,
              double* Q, int ldq, int block, bdc_stream_t stream);

/* ---- launch tuning ---------------------------------------------------------
 * Launch shapes of the vector-update products.  The autotuner times a small
 * set of candidates on the caller's own problem (or batch) and keeps the
 * fastest in the handle; results satisfy the same tolerances with any
 * tuning. */
typedef struct {
  int small_n;  /* merges with at most this many kept values use 64 x 64 output
                   tiles, larger ones 128 x 128 (32..2^20; default 96; at or
                   above the largest merge, no 128 x 128 launch at all) */
  int flat;     /* 1: all tiles of a merge level in one flattened list walked by a
                   persistent grid; 0 (default): a grid slice per merge */
  int grid64;   /* workgroups of the 64-tile product (flat), or half the per-merge cap */
  int grid128;  /* the same for the 128-tile product */
  int sec_small_n; /* secular problems with at most this many roots (0..256;
                      default 256) are solved with 8 or 16 lanes per root and no
                      workgroup barriers; larger ones with one lane per root and
                      the poles split over four wavefronts */
  int leaf_size;   /* the tree's leaf size (4..32; 0 in bdc_set_tuning keeps the
                      handle's); the paper found 32 best on its GPUs */
  int tile128;     /* 128 x 128 products with a grid per merge: 0 a
                      single-buffered LDS tile, 1 (default) a double-buffered
                      tile at two workgroups per CU (bitwise the same sums) */
  int streams;     /* 1 (default): every launch of a solve on one stream; 2:
                      each level's rotations and gather of the kept columns
                      run on a second stream beside its secular solve, Löwner
                      z and vectors (captured solves only; the same results).
                      Pays where the gathers are long (batches of undeflated
                      merges); costs a few microseconds per level where every
                      launch is short */
  float ms;     /* out (bdc_autotune): time per solve of the chosen tuning */
} bdc_tuning_t;

int bdc_get_tuning(bdc_handle_t handle, bdc_tuning_t* tuning);
int bdc_set_tuning(bdc_handle_t handle, const bdc_tuning_t* tuning);
/* Times candidate tunings on bdc_svd_batched(batch, sizes, d, e, sigma, U,
 * VT) (arguments as there; a single problem is batch = 1): one warm-up and
 * `repeats` timed solves each, with HIP events on `stream`; first the leaf
 * size (8, 12, 16, 20, 24, 32), then the launch shapes with the best one, then
 * the other 128 x 128 tile and the other stream count.  Keeps the
 * fastest in the handle and returns it in *best.  Synchronous: waits for the
 * stream.  The outputs hold the last solve's results. */
int bdc_autotune(bdc_handle_t handle, int64_t batch, const int64_t* sizes, const double* d,
                 const double* e, double* sigma, double* U, double* VT, bdc_stream_t stream,
                 int repeats, bdc_tuning_t* best);

/* ---- learned start of the secular iteration ------------------------------
 * The paper solves each secular equation with LAPACK's lasd4; this library
 * adds an optional learned first point: a 19 -> 64 -> 64 -> 64 -> 1 MLP
 * (GELU hidden layers, logistic output) maps the features above to the
 * root's fractional position in its interval.  Its hidden-layer products run
 * on bfloat16 matrix cores with FP32 accumulation: every product operand
 * (inputs, weights, activations and, in training, back-propagated gradients)
 * is rounded to bfloat16; everything else is FP32.  Parameters: one FP32
 * vector of BDC_MLP_PARAMS numbers, W1 (19 x 64 row-major, in x out), b1
 * (64), W2 (64 x 64), b2, W3 (64 x 64), b3, W4 (64), b4 (1).  The network is
 * owned by the handle; training updates it in place. */

/* Copy host parameters into the handle (synchronous); resets Adam's state. */
int bdc_mlp_set(bdc_handle_t handle, const float* params, int64_t count);
/* Copy the handle's parameters to the host (waits for the handle's stream). */
int bdc_mlp_get(bdc_handle_t handle, float* params, int64_t count);
/* xhat (device, rows floats) = network(X) for X (device, rows x 19). */
int bdc_mlp_forward(bdc_handle_t handle, const float* X, int64_t rows, float* xhat,
                    bdc_stream_t stream);
/* Gradient (device, BDC_MLP_PARAMS floats) and, if loss != NULL, the loss
 * (device, 1 float) of the mean squared error of network(X) against y
 * (device, rows floats) over the rows; 1 <= rows <= 2^24. */
int bdc_mlp_grad(bdc_handle_t handle, const float* X, const float* y, int64_t rows, float* grad,
                 float* loss, bdc_stream_t stream);
/* `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr)
 * on the mean squared error; step s uses rows idx[s*batch .. s*batch+batch)
 * of (X, y) (device int32 row indices).  loss_hist (device, steps floats,
 * may be NULL) receives each step's batch loss before its update. */
int bdc_mlp_train(bdc_handle_t handle, const float* X, const float* y, const int32_t* idx,
                  int64_t batch, int64_t steps, float lr, float* loss_hist, bdc_stream_t stream);
/* Collect training rows from later solves on this handle: after each merge's
 * secular solve, every root appends its features (X, rows x 19), the
 * position of the computed root in its interval (y) and a tag (3 int32:
 * problem offset + node's first row, node rows, root index).  The row counter
 * *count (device, uint64; the caller zeroes it) is advanced by every root;
 * rows past `capacity` are not written.  Solves run without graph replay
 * while collecting.  X = NULL stops collecting. */
int bdc_set_harvest(bdc_handle_t handle, float* X, float* y, int32_t* tag, int64_t capacity,
                    unsigned long long* count);

/* C (M x N, ldc) = A (M x K, lda) * B (K x N, ldb), column-major FP64, through
 * the split-precision kernels of BDC_GEMM_OZAKI with `slices` slices (5..7):
 * every row of A and column of B scaled by a power of two and cut into 8-bit
 * digits held exactly in bfloat16, digit products with p + q <= slices - 1
 * summed on the bfloat16 matrix cores in FP32 (exactly for the three leading
 * weights) and combined in FP64. */
int bdc_step_gemm_ozaki(bdc_handle_t handle, int slices, int M, int N, int K, const double* A, int lda,
                        const double* B, int ldb, double* C, int ldc, bdc_stream_t stream);

/* C (M x N, ldc) = A (M x K, lda) * B (K x N, ldb), column-major FP64, on
 * the int8 matrix cores through the Chinese remainder theorem (the
 * integer-modular emulation known as Ozaki scheme II): every row of A and
 * column of B is scaled by a power of two and rounded to an integer; the
 * integer product is formed exactly from its residues modulo `moduli`
 * (13..16) pairwise coprime odd moduli <= 255, each an int8 x int8 -> int32
 * product, and rebuilt by Garner's mixed-radix algorithm.  The scale is the
 * largest one for which the rebuilt product is exact (K <= 2^20), so the
 * error comes only from rounding A and B at about 2^-beta of each row's /
 * column's largest entry, beta = min(55, floor((log2 prod m - 1 - log2 K) / 2))
 * (54 with 16 moduli and K = 16384), plus the single final rounding to FP64
 * (the integer is rebuilt exactly, so exact integer products come out bit
 * for bit). */
int bdc_step_gemm_crt(bdc_handle_t handle, int moduli, int M, int N, int K, const double* A, int lda,
                      const double* B, int ldb, double* C, int ldc, bdc_stream_t stream);

const char* bdc_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* BDC_H_ */
