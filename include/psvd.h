/*
 * psvd.h -- C ABI of the MI355X (gfx950) streaming / randomized / partitioned
 * SVD library, after Maulik & Mengaldo, "PyParSVD: a streaming, distributed
 * and randomized singular-value-decomposition library" (arXiv 2108.08845).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrices are column-major: element (i, j) of a matrix with leading
 *    dimension ld is at base[i + j*ld]; each snapshot (column) is contiguous.
 *    A contiguous torch tensor of shape (N, M) is the M x N matrix.
 *  - Device pointers are HIP device memory owned by the caller unless stated
 *    otherwise; host pointers are ordinary host memory.
 *  - All device work is enqueued on the stream given at creation (NULL: the
 *    default stream).  Calls that return host data synchronise that stream.
 *  - Return value: PSVD_OK (0) or a negative psvd_status.  No exception
 *    crosses the ABI.  A failed call leaves the handle's state unchanged; the
 *    text of the last error is available from psvd_last_error().
 *  - Errors detected on the device (non-finite data, a step that cannot
 *    proceed) are reported by the call that detects them; with
 *    PSVD_OPT_ASYNC set they surface at the next synchronising call.
 *  - One handle is used by one host thread at a time.
 */
#ifndef PSVD_H
#define PSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct psvd_handle psvd_handle;

typedef enum psvd_status {
    PSVD_OK = 0,
    PSVD_E_INVAL = -1,      /* invalid argument value                            */
    PSVD_E_SHAPE = -2,      /* inconsistent sizes / leading dimensions           */
    PSVD_E_DTYPE = -3,      /* unsupported element type for this precision       */
    PSVD_E_NOMEM = -4,      /* device or host allocation failed                  */
    PSVD_E_NONFINITE = -5,  /* NaN or Inf reached the small factorisations       */
    PSVD_E_NOCONV = -6,     /* Jacobi SVD did not converge within max_sweeps     */
    PSVD_E_BREAKDOWN = -7,  /* Cholesky breakdown with the fallback disabled      */
    PSVD_E_DEVICE = -8,     /* HIP runtime error                                 */
    PSVD_E_STATE = -9       /* call not valid in the handle's current state      */
} psvd_status;

typedef enum psvd_dtype { PSVD_F32 = 1, PSVD_F64 = 2 } psvd_dtype;

typedef enum psvd_method {
    PSVD_DETERMINISTIC = 0, /* QR of the panel + SVD of R (Algorithm 1)          */
    PSVD_RANDOMIZED = 1     /* randomized range finder on the panel (Eqs. 7-11)  */
} psvd_method;

typedef enum psvd_precision {
    PSVD_PREC_FP64 = 0,     /* every product in FP64; state U in FP64            */
    PSVD_PREC_FP32 = 1,     /* panel products in FP32 (MFMA), small core FP64    */
    PSVD_PREC_MIXED = 2,    /* power passes FP32-accurate on the BF16 matrix
                               cores: every operand split into three BF16 terms,
                               six term products with FP32 accumulation; the final
                               projection with every operand split into a BF16
                               pair (hi + lo); Grams summed in FP64, small core
                               FP64; lift FP32                                  */
    PSVD_PREC_BF16 = 3      /* power passes on plain BF16 operands (the
                               unrefined sketch), the final projection as in
                               MIXED but with a BF16-rounded test matrix: faster,
                               with the BF16 sketch's error                      */
} psvd_precision;

enum {
    PSVD_OPT_ASYNC = 1,        /* do not synchronise at the end of each update     */
    PSVD_OPT_NO_FALLBACK = 2,  /* report Cholesky breakdown instead of falling back */
    PSVD_OPT_PROFILE = 4,      /* time each tall-panel kernel with HIP events      */
    PSVD_OPT_OMEGA_BF16 = 8,   /* test matrices rounded to BF16 values whatever the
                                  precision (the values MIXED and BF16 use), so
                                  precisions can be compared on identical ones    */
    PSVD_OPT_GRAPH = 16        /* launch a randomized update's kernels as one
                                  hipGraph (captured on a stream of the library,
                                  updated in place while only arguments change)
                                  instead of one by one; not with PSVD_OPT_PROFILE */
};

/* Kernel classes timed with PSVD_OPT_PROFILE (index into psvd_stats_t arrays). */
enum {
    PSVD_KC_FUSED_BF16 = 0,    /* C^T (C X) in BF16 (power passes, BF16 precision) */
    PSVD_KC_FUSED_F32 = 1,     /* C^T (C X) [and (C X)^T (C X)] on the FP32 matrix
                                  cores (power passes and final pass of FP32)      */
    PSVD_KC_LIFT = 2,          /* U <- C T                                         */
    PSVD_KC_TN = 3,            /* reductions over the tall rows (Gram, C^T Y)     */
    PSVD_KC_NN = 4,            /* other tall products (C X written out)           */
    PSVD_KC_SMALL = 5,         /* small-core kernels without an SVD (Cholesky-QR) */
    PSVD_KC_SMALL_SVD = 6,     /* small-core kernels with the one-sided Jacobi SVD */
    PSVD_KC_SPLIT = 7,         /* final passes on split-BF16 operands (C^T Y, Y kept) */
    PSVD_KC_SPLIT3 = 8,        /* C^T (C X) on three-term BF16 splits: the FP32-
                                  accurate power passes of the mixed precision     */
    PSVD_KC_WIDE = 9,          /* C X and C^T Y on the FP32 matrix cores for panels
                                  wider than the fused passes take, one read of
                                  the panel per product                            */
    PSVD_KC_COUNT = 10
};

typedef struct psvd_options {
    int32_t method;         /* psvd_method                                       */
    int32_t precision;      /* psvd_precision                                    */
    uint64_t seed;          /* key of the Gaussian test matrices                 */
    void* stream;           /* hipStream_t; NULL = default stream                */
    int32_t max_sweeps;     /* Jacobi sweep limit (default 60)                   */
    int32_t flags;          /* PSVD_OPT_* bits                                   */
    int32_t tile_rows;      /* fused passes: row-tile height 16/32/64, 0 = default */
    int32_t wg_per_cu;      /* fused passes: work-groups per compute unit 1..4,
                               0 = default (1); see the autotuner               */
    int32_t panel_width;    /* fused passes: plan for a panel at least this wide
                               (a wider compiled tile width), 0 = the panel's   */
    int32_t split_m;        /* generic tall products: work items the rows are
                               split into (times output blocks), 0 = 1024       */
} psvd_options;

typedef struct psvd_stats_t {
    int64_t batches;            /* updates applied                               */
    int64_t fallbacks;          /* Cholesky breakdowns handled by the eigen route */
    int32_t last_sweeps;        /* Jacobi sweeps of the last small SVD           */
    int32_t last_path;          /* 0 deterministic, 1 randomized                 */
    double last_update_ms;      /* device time of the last update (events)       */
    int64_t kernel_launches[10]; /* per kernel class (PSVD_OPT_PROFILE)          */
    double kernel_ms[10];        /* summed device time per kernel class          */
} psvd_stats_t;

/* Fill *opt with defaults: deterministic, FP64, seed 0, default stream. */
void psvd_default_options(psvd_options* opt);

/*
 * Create a streaming-SVD state for snapshots of M rows keeping K modes
 * (Algorithm 1 of Sec. 3.1: forget factor ff weights the previous modes,
 * 0 < ff <= 1).  oversampling p and power_iters q configure the randomized
 * range finder of Sec. 3.3 (sketch width K + p).  The state starts empty
 * (rank r = 0).  The library owns U (M x K, double-buffered), the singular
 * values and all workspace.  Errors: PSVD_E_INVAL (K < 1, K > M, ff outside
 * (0, 1], p < 0, q < 0, unknown method/precision), PSVD_E_NOMEM.
 */
int psvd_initialize(psvd_handle** h, int64_t M, int32_t K, double ff, int32_t oversampling, int32_t power_iters,
                    const psvd_options* opt);

/*
 * Ingest one batch A (M x N, device, column-major, leading dimension
 * lda >= M, element type dtype).  With r = 0 this is the initialisation
 * (the initialisation of Algorithm 1: factor A alone); otherwise the update on the
 * panel [ff * U diag(s) | A].  Deterministic method: tall-skinny QR of the
 * panel (Cholesky-QR twice, eigen route on breakdown), one-sided Jacobi SVD
 * of R, keep K, U <- Q U~_K.  Randomized method with K + p < r + N: sketch
 * Y = panel * Omega with the batch's Gaussian test matrix, q power
 * iterations, projection B = Q^T panel, Jacobi SVD of B, U <- Q U~_K
 * (Eqs. 7-11); otherwise the deterministic step.  Afterwards
 * r = min(K, r + N).  A is read on the handle's stream and must stay valid
 * until the stream passes this call.  N = 0 is a no-op.
 * Errors: PSVD_E_SHAPE (M mismatch, lda < M, r + N > M), PSVD_E_DTYPE
 * (PSVD_F64 data with a non-FP64 precision), PSVD_E_NONFINITE, PSVD_E_NOCONV,
 * PSVD_E_BREAKDOWN, PSVD_E_DEVICE.
 */
int psvd_incorporate_data(psvd_handle* h, const void* A, int64_t M, int64_t N, int64_t lda, int32_t dtype);

/* Current rank r (0 before the first batch). */
int psvd_rank(const psvd_handle* h, int32_t* r);

/*
 * Copy the r singular values (descending, FP64) to host memory out
 * (capacity cap >= r); *r receives the rank.  Synchronises the stream.
 */
int psvd_singular_values(const psvd_handle* h, double* out, int32_t cap, int32_t* r);

/*
 * Copy the M x r modes U into caller device memory (leading dimension
 * ldu >= M) converted to dtype.  Enqueued on the handle's stream.
 */
int psvd_modes(const psvd_handle* h, void* U, int64_t ldu, int32_t dtype);

/*
 * Borrowed pointer to the library's current U (M x r, column-major, leading
 * dimension *ldu, element type *dtype).  Valid until the next update or
 * psvd_finalize.
 */
int psvd_modes_ptr(const psvd_handle* h, const void** U, int64_t* ldu, int32_t* dtype);

/*
 * The Gaussian test matrix the handle uses for update number `batch` on a
 * panel of n columns (n x (K + p), column-major, FP64 values exactly as the
 * device consumes them) -- Sec. 3.3's random matrix, from the counter-based
 * generator Philox4x32-10 (Salmon et al., SC'11) keyed by (seed, batch) and
 * Box-Muller, rounded to the precision's input type.  out: host memory.
 */
int psvd_get_omega(const psvd_handle* h, int64_t batch, int64_t n, double* out);

/*
 * Launch parameters of the tall-panel kernels (the fields tile_rows, wg_per_cu,
 * panel_width and split_m of psvd_options, with the same meaning and ranges),
 * set on an existing handle, e.g. from an autotuner's cache once the batch
 * width is known.  They change the grouping of the fixed-order partial sums
 * (results agree to rounding), not what is computed.  Errors: PSVD_E_INVAL.
 */
int psvd_set_tuning(psvd_handle* h, int32_t tile_rows, int32_t wg_per_cu, int32_t panel_width, int32_t split_m);

/* Metrics of the handle (host copy); synchronises the stream when profiling. */
int psvd_stats(const psvd_handle* h, psvd_stats_t* out);

/* Zero the counters of psvd_stats (not the state). */
int psvd_reset_stats(psvd_handle* h);

/*
 * Checkpoint of the streaming state (Algorithm 1 carries U, s and the batch
 * count from one update to the next; nothing else is needed to resume).
 * psvd_save_state writes a self-describing host buffer: a header with the
 * configuration (M, K, ff, p, q, method, precision, seed), the rank r and
 * the batch count, then K FP64 singular values (zero beyond r) and the r
 * columns of U (M values each, in the state's element type).  buf == NULL
 * only reports the size in *size.  Synchronises the stream.
 * Errors: PSVD_E_INVAL (cap smaller than the state), PSVD_E_DEVICE.
 *
 * psvd_load_state restores such a buffer into a handle created with the same
 * configuration; the next update then draws the Gaussian test matrix of the
 * restored batch count, so a resumed stream reproduces the uninterrupted one
 * bit for bit.  Errors: PSVD_E_INVAL (not a state buffer, truncated),
 * PSVD_E_STATE (different configuration); the state is unchanged on error.
 */
int psvd_save_state(const psvd_handle* h, void* buf, size_t cap, size_t* size);
int psvd_load_state(psvd_handle* h, const void* buf, size_t size);

/*
 * One-shot randomized SVD of one matrix (Sec. 3.3, Eqs. 7-11): the sketch
 * Y = A Omega with an (N x (K+p)) Gaussian test matrix drawn from (seed,
 * batch 0), q power iterations, B = Q^T A, B = U~ S V~^T, U = Q U~[:, :K],
 * V = V~[:, :K], computed as one update of an empty randomized stream (the
 * exact SVD when K + p >= N).  A: device, M x N, leading dimension lda,
 * a_dtype (PSVD_F64 data needs PSVD_PREC_FP64).  Outputs (each may be NULL):
 * U device M x rank (ldu, out_dtype); V device N x rank (ldv, out_dtype),
 * V = A^T U diag(1/s); s host, K values; *rank = min(K, N).  Synchronises.
 * Errors: PSVD_E_INVAL, PSVD_E_SHAPE, PSVD_E_DTYPE, PSVD_E_NOMEM,
 * PSVD_E_NONFINITE, PSVD_E_DEVICE; the text is psvd_last_error(NULL).
 */
int psvd_rsvd(const void* A, int64_t M, int64_t N, int64_t lda, int32_t a_dtype, int32_t K, int32_t oversampling,
              int32_t power_iters, uint64_t seed, int32_t precision, void* U, int64_t ldu, void* V, int64_t ldv,
              int32_t out_dtype, double* s, int32_t* rank, void* stream);

/*
 * psvd_rsvd without any allocation, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same computation, arguments and results as
 * psvd_rsvd, with every piece of device workspace taken from a fixed array
 * of PSVD_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until
 * the process ends, and fixed host buffers (a test matrix of at most
 * PSVD_NOALLOC_OMEGA_ENTRIES = N x (K + p) entries).  The call allocates
 * nothing: no hipMalloc, hipFree or other allocating routine.  U (if not NULL)
 * must have out_dtype = the precision's element type (PSVD_F64 for
 * PSVD_PREC_FP64, PSVD_F32 otherwise); the modes are written into it directly.
 * The workspace grows with M (K + p) (the kept sketch) plus the partial sums;
 * a problem that needs more than the fixed array returns PSVD_E_NOMEM with the
 * required size in psvd_last_error(NULL).  Calls of one process are
 * serialised by a lock and each synchronises the stream before it returns;
 * work of another caller left on the array is overwritten (calls that
 * overlapped on one GPU -- impossible within a process -- would race).
 * Errors: those of psvd_rsvd, plus PSVD_E_DTYPE (U element type) and
 * PSVD_E_NOMEM (size beyond the fixed maximum).
 */
#define PSVD_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
#define PSVD_NOALLOC_OMEGA_ENTRIES ((size_t)1 << 20)
int psvd_rsvd_noalloc(const void* A, int64_t M, int64_t N, int64_t lda, int32_t a_dtype, int32_t K,
                      int32_t oversampling, int32_t power_iters, uint64_t seed, int32_t precision, void* U,
                      int64_t ldu, void* V, int64_t ldv, int32_t out_dtype, double* s, int32_t* rank, void* stream);

/* Text of the last error on this handle ("" if none).  Owned by the handle.
 * With h == NULL: the last error of a psvd_rsvd call on this host thread. */
const char* psvd_last_error(const psvd_handle* h);

/* Static name of a status code. */
const char* psvd_status_string(int status);

/* Release the handle and everything it owns (NULL is allowed). */
void psvd_finalize(psvd_handle* h);

/*
 * Approximate partitioned method of snapshots (Algorithm 2, Eqs. 3-6) over P
 * row partitions of one data set, all on this GPU, in one enqueued sequence:
 *   1. G_i = A_i^T A_i (method of snapshots, the option of Sec. 3.2) and its
 *      eigen-decomposition by one-sided Jacobi -> V_i, sigma_i;
 *   2. W_i = V_i[:, :r] diag(sigma_i[:r]);  W = [W_1 ... W_P]  (N x P r);
 *   3. W = X Lambda Y^T;  X~ = X[:, :K], Lambda~ = Lambda[:K];
 *   4. U_i = A_i X~ diag(1 / Lambda~).
 * A_parts[i]: device, M_parts[i] x N, leading dimension ld_parts[i] >= M_i,
 * element type dtype (PSVD_F32 or PSVD_F64).  U_parts[i]: device output
 * M_parts[i] x K (leading dimension ldu_parts[i], same dtype).  Lambda (K)
 * and X (N x K, column-major) are host outputs (may be NULL).  Pointer
 * arrays are host arrays.  Synchronises the stream.
 * Errors: PSVD_E_INVAL (P < 1, r < 1, r > N, K < 1, K > min(N, P r),
 * Lambda~_K <= N 2^-53 Lambda~_1), PSVD_E_SHAPE, PSVD_E_NOCONV, PSVD_E_NOMEM,
 * PSVD_E_DEVICE.
 */
int psvd_apmos_batched(int32_t P, const void* const* A_parts, const int64_t* M_parts, const int64_t* ld_parts,
                       int64_t N, int32_t dtype, int32_t r, int32_t K, void* const* U_parts,
                       const int64_t* ldu_parts, double* Lambda, double* X, void* stream);

/*
 * Algorithm 2 as psvd_apmos_batched, with the SVD of W in step 3 taken by the
 * low-rank SVD of Sec. 3.3 (Eqs. 7-11 without power iterations): Y = W Om
 * with the Gaussian test matrix Om (P r x ell, FP64 values of the generator of
 * psvd_get_omega keyed by (seed, 0)), Q = orth(Y), B = Q^T W = U~ S V~^T,
 * X~ = Q U~[:, :K], Lambda~ = S[:K] -- where the paper's parallel listing
 * randomizes.  K <= ell <= min(N, P r).  Exact when rank(W) <= ell.
 * Arguments, outputs and errors as psvd_apmos_batched.
 */
int psvd_apmos_low_rank(int32_t P, const void* const* A_parts, const int64_t* M_parts, const int64_t* ld_parts,
                        int64_t N, int32_t dtype, int32_t r, int32_t K, int32_t ell, uint64_t seed,
                        void* const* U_parts, const int64_t* ldu_parts, double* Lambda, double* X, void* stream);

/*
 * Partitioned streaming: the parallel streaming SVD of Section 3 (the
 * initialisation by APMOS, Algorithm 2, and the batch update with a QR over
 * row partitions) with P row partitions of the data, all on this GPU.
 * M_parts[i] >= 1 rows per partition; K modes; ff in (0, 1]; r_local the
 * local truncation of the APMOS initialisation (0: min(K, N)).  opt:
 * PSVD_PREC_FP64 (FP64 data and state) or PSVD_PREC_FP32 (FP32 data and
 * state); method PSVD_DETERMINISTIC takes exact SVDs of W and of the combined
 * R factor, PSVD_RANDOMIZED the paper's placement of randomization in the
 * parallel variant: both by the low-rank SVD of Sec. 3.3 (Eqs. 7-11) with a
 * K-column Gaussian test matrix, FP64 values keyed by (opt.seed, b) for batch
 * b (the initialisation is batch 0).  The handle works with
 * psvd_pstream_incorporate / psvd_pstream_modes_ptr and psvd_rank,
 * psvd_singular_values, psvd_stats, psvd_last_error, psvd_finalize; the
 * single-panel calls (incorporate_data, modes, checkpoints) return
 * PSVD_E_STATE on it.
 * Errors: PSVD_E_INVAL (P < 1, M_i < 1, K < 1, K > sum M_i, ff, options),
 * PSVD_E_NOMEM, PSVD_E_DEVICE.
 */
int psvd_pstream_initialize(psvd_handle** h, int32_t P, const int64_t* M_parts, int32_t K, double ff,
                            int32_t r_local, const psvd_options* opt);

/*
 * One batch of N columns, partition i in A_parts[i] (device, M_i x N,
 * leading dimension ld_parts[i] >= M_i, element type dtype = the state's).
 * First batch (rank 0): APMOS over the partitions (needs K <= N and
 * r_local <= N), U_i = A_i X~ diag(1 / Lambda~), s = Lambda~.  Later
 * batches: panels C_i = [ff U_i diag(s) | A_i] (M_i >= r + N rows each), the
 * R factor of the stacked panel from the partitions' Gram sum (the R factor
 * of the stacked local R factors), Jacobi SVD of R with the stable
 * descending sort and sign rule of Algorithm 1, U_i = C_i R^-1 U~_K, kept
 * rank min(K, r + N).  Host pointer arrays; synchronises the stream.
 * Errors: PSVD_E_STATE (not a partitioned handle), PSVD_E_INVAL, PSVD_E_SHAPE,
 * PSVD_E_DTYPE, PSVD_E_NONFINITE, PSVD_E_NOCONV, PSVD_E_NOMEM, PSVD_E_DEVICE;
 * on error the state is unchanged.
 */
int psvd_pstream_incorporate(psvd_handle* h, const void* const* A_parts, const int64_t* ld_parts, int64_t N,
                             int32_t dtype);

/* Borrowed pointer to partition part's modes (M_part x rank, leading dimension
 * *ldu = M_part, element type *dtype), valid until the next mutating call. */
int psvd_pstream_modes_ptr(const psvd_handle* h, int32_t part, const void** U, int64_t* ldu, int32_t* dtype);

/* Copy of partition part's modes into U (device, M_part x rank, leading
 * dimension ldu >= M_part, the state's element type), stream-ordered. */
int psvd_pstream_modes(const psvd_handle* h, int32_t part, void* U, int64_t ldu);

/*
 * Reverse-mode derivative of the deterministic stream (Algorithm 1 with the
 * QR + SVD(R) step) over B equal batches of Nb columns of A (device,
 * M x B*Nb, leading dimension lda, dtype) with K modes and forget factor ff:
 * given cotangents U_bar (device, M x r, leading dimension M, dtype) of the
 * final modes and s_bar (host, r values) of the final singular values,
 * writes A_bar (device, M x B*Nb, leading dimension M, dtype).  Each batch's
 * panel is recomputed from the stored incoming state (memory O(M K) per
 * batch) and the adjoint of its thin SVD is applied,
 *   C_bar = U [diag(s_bar) + (F o (U^T U_bar - U_bar^T U)) S] V^T
 *           + (I - U U^T) U_bar S^-1 V^T,   F_ij = 1 / (s_j^2 - s_i^2),
 * with F used only for pairs that touch a retained index and guarded at
 * near-degenerate pairs.  Synchronises the stream.
 */
int psvd_stream_backward(const void* A, int64_t M, int64_t lda, int32_t dtype, int32_t B, int64_t Nb, int32_t K,
                         double ff, const void* U_bar, const double* s_bar, void* A_bar, void* stream);

/*
 * Loss of the streamed truncated SVD and its gradient, entirely on the
 * device: L = ||A - U U^T A||_F^2 + sum_{j<r} w_j s_j, with (U, s) the
 * deterministic stream over B batches of Nb columns (K modes, ff), the
 * residual evaluated as ||A||^2 - sum_b ||U^T A_b||^2.  w: host, K weights.
 * loss: host scalar (may be NULL).  grad: device M x B*Nb (leading
 * dimension M, dtype), may be NULL for the loss alone.  Synchronises.
 */
int psvd_loss_grad(const void* A, int64_t M, int64_t lda, int32_t dtype, int32_t B, int64_t Nb, int32_t K,
                   double ff, const double* w, double* loss, void* grad, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PSVD_H */
