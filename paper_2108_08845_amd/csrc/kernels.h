// kernels.h -- argument blocks and launchers of the device kernels.
#pragma once

#include "psvd_internal.h"

namespace psvd {

constexpr int TN_OB = 64;   // output block edge of k_tn
constexpr int FU_LB = 64;   // sketch columns per work-group of k_fused
constexpr int FU_MAX_WG = 1024;   // work-groups per column block of a fused pass (4 per CU)

// Output block y of a blocked product -> (block row, block col).
__host__ __device__ inline void block_coords(int y, int mbl, int sym, int* bi, int* bj) {
    if (!sym) {
        *bi = y % mbl;
        *bj = y / mbl;
        return;
    }
    int j = 0;
    while ((j + 1) * (j + 2) / 2 <= y) ++j;
    *bj = j;
    *bi = y - j * (j + 1) / 2;
}

// Row chunk (a multiple of 64) splitting segments of the given row counts, each
// on its own, into at most `target` work items: the smallest such chunk (one
// item per segment when there are more segments than that).
inline int64_t chunk_for_items(const int64_t* rows, int nseg, int64_t target) {
    int64_t total = 0, most = 64;
    for (int i = 0; i < nseg; ++i) {
        total += rows[i];
        most = rows[i] > most ? rows[i] : most;
    }
    int64_t chunk = ((total + target - 1) / (target > 0 ? target : 1) + 63) / 64 * 64;
    chunk = chunk < 64 ? 64 : chunk;
    for (;; chunk += 64) {
        int64_t cnt = 0;
        for (int i = 0; i < nseg; ++i) cnt += (rows[i] + chunk - 1) / chunk;
        if (cnt <= target || chunk >= most) return chunk;
    }
}

struct TnArgs {
    PanelSeg lseg, rseg;     // single-segment operands (used when lsegs == nullptr)
    const PanelSeg* lsegs;   // L operand segments (device array) or nullptr
    const PanelSeg* rsegs;   // R operand segments
    const WorkItem* items;   // explicit work items or nullptr: item i = rows [i*chunk, (i+1)*chunk)
    int64_t chunk;
    int32_t mbl;             // output blocks along the rows of the result (ceil(nl / 64))
    int32_t sym;             // only blocks (i <= j) are computed
    double* part;            // [item][ob] 64 x 64 column-major FP64
    const int32_t* skip;     // if non-null and *skip & skip_mask: do nothing
    int32_t skip_mask;
    int32_t nob;
    int32_t nitems;          // work items (set by launch_tn)
    int32_t vec;             // 16-byte column loads (k_tn_v): every block of both operands
                             //   16-byte aligned, leading dimensions, segment rows and item
                             //   row ranges multiples of 4
    int32_t dtype_all;       // PSVD_F32 / PSVD_F64 when every column of both operands (every
                             //   segment) has that dtype, else 0 (k_tn_w needs one)
};

struct TnReduceArgs {
    const double* row_scale;    // output rows gi < nscale multiplied by row_scale[gi] (not with sym)
    int32_t nscale;
    const double* part;
    const int32_t* seg_item0;   // first item of each segment (size nseg + 1), or nullptr: items [0, nitems)
    int32_t nitems;
    int32_t mbl;
    int32_t nob;
    int32_t nl, nr;
    int32_t sym;
    double* out;                // nseg consecutive nl x nr matrices
    const int32_t* skip;
    int32_t skip_mask;
};

struct NnArgs {
    PanelSeg seg;        // single segment (used when segs == nullptr)
    const PanelSeg* segs;
    const WorkItem* items;
    int64_t chunk;
    const double* row_scale;  // optional: output row i < nscale multiplied by row_scale[i]
    int32_t nscale;
    const double* X;     // n x nx, column-major, ld ldx (shared by all segments)
    int64_t ldx;
    int32_t n;           // rows of X used (= panel columns)
    int32_t nx;          // output columns
    const int32_t* skip;
    int32_t skip_mask;        // do nothing if (*skip & skip_mask)
    int32_t need_mask;        // do nothing unless (*skip & need_mask) (when non-zero)
    int32_t accumulate;       // out += result instead of out = result
    int32_t all_f32;          // every segment's columns FP32 (k_nn_v)
    int32_t vec_f32;          // ... and float4-aligned (rows % 4 == 0, 16-byte column starts)
    int32_t nitems_v;         // work items (set by the launcher)
    int32_t vec16;            // every block 16-byte aligned, leading dimensions, rows and item
                              //   row ranges multiples of 4 (k_nn_w)
};

struct FusedArgs {
    PanelSeg seg;            // panel (FP32 blocks)
    const double* X;         // n x lx, ld ldx (logical operand, already scaled)
    int64_t ldx;
    int32_t n, np;           // panel columns; np = the kernel's padded width (FusedPlan)
    int32_t lx;              // columns of X
    int32_t nlb;             // column blocks (ceil(lx / 64))
    int32_t tm;              // rows per tile (FusedPlan)
    int32_t nwg;             // work-groups per column block
    int64_t tiles;           // ceil(rows / tm)
    float* partP;            // [wg][lb] np x 64 column-major
    double* partG;           // [wg] 64 x 64 (only when nlb == 1 and G requested)
    int32_t want_g;          // FP32 compute type only
    int32_t vec;             // float4 loads/stores allowed (rows % 4 == 0, lds % 4 == 0, 16-byte bases)
    float* yout;             // final pass: optional copy of Y = C X (rows x lx, ld ldy)
    int64_t ldy;
};

struct FusedReduceArgs {
    const double* row_scale;   // P rows i < nscale multiplied by row_scale[i] (may be null)
    int32_t nscale;
    const float* partP;
    const double* partG;
    int32_t nwg, nlb, np, n, lx;
    int32_t want_g;
    double* P;
    double* G;
};

struct SmallArgs {
    int32_t n;            // panel columns r + N
    int32_t r;            // current rank (columns of the U part)
    int32_t K;
    int32_t l;            // sketch width (randomized)
    int32_t max_sweeps;
    int32_t allow_fallback;
    const double* d;      // d[j] = ff * s_j, j < r (column scale of the U part)
    double* G;            // n x n (deterministic Gram, then work)
    double* G2;           // n x n
    double* R1;           // n x n
    double* Ri;           // n x n
    double* Z;            // n x n Jacobi work
    double* T;            // n x K  (lift operand, already scaled by D)
    double* Xn;           // n x n  (pass-2 operand D R1^-1)
    double* s_out;        // K new singular values
    double* small_u;      // n x K small left factor after the sign rule (diagnostics)
    double* vec;          // 4n scratch
    int32_t* ivec;        // 3n scratch
    int32_t* status;      // DevStatus bits
    int32_t* sweeps;      // last Jacobi sweep count
    int32_t skip_svd;     // k_small_det2 stops after R = R2 R1 (the caller takes the SVD of R)
    double stop_cos2;     // > 0: the Jacobi of R ends after a sweep whose largest cos^2 is at
                          //   most max(this, m 2^-53) (FP32 precision); 0: no early end
};

struct OrthArgs {
    int32_t n, l;
    const double* P;      // n x l (ld n)
    double* G;            // l x l scratch: P^T P (kept for the shifted retry)
    double* R;            // l x l scratch (used when the factors do not fit in LDS)
    double* Ri;           // l x l scratch (same)
    double* vec;          // 4 l scratch (same)
    double* X;            // n x l out (ld n): D P R^-1
    const double* d;      // row scale d[i], i < r
    int32_t r;
    int32_t* status;
    int32_t flag_bit;     // status bit set on a shifted retry
};

struct RandFinalArgs {
    int32_t n, l, K;
    int32_t max_sweeps;
    double stop_cos2;     // Jacobi (l <= 64) ends after a sweep with largest cos^2 <= this (0: m 2^-53)
    int32_t qr_passes;    // Cholesky-QR passes for the R factor of P (2, or 1 in the mixed precision)
    const double* P;      // n x l (ld n): C^T Y
    double* P1;           // n x l scratch: P R1^-1
    const double* GY;     // l x l: Y^T Y
    double* RY;           // l x l out: chol(Y^T Y)
    double* RYi;          // l x l out: R_Y^-1
    double* G1;           // l x l scratch: P^T P
    double* R1;           // l x l scratch: chol(P^T P)
    double* W;            // l x l scratch (used when the factors do not fit in LDS)
    double* V;            // l x l scratch (same)
    double* vec;          // 4 l scratch (same)
    double* M2;           // l x K out: R_Y^-1 U~_K
    double* s_out;        // K
    double* small_u;      // l x K
    int32_t* status;
    int32_t* sweeps;
};

struct ApmosLocalArgs {
    double* G;          // P consecutive N x N Grams (destroyed)
    double* Wt;         // (P r) x N, column-major: row block i = W_i^T
    int32_t N, r, P;
    int32_t max_sweeps;
    int32_t data_f32;   // partitions stored in FP32: the eigen-decompositions' rank
                        //   tolerance is the data's rounding level (N 2^-48 max diag)
    double* vec;        // P * 2N
    int32_t* ivec;      // P * 3N
    int32_t* status;
    int32_t* sweeps;
};

struct ApmosGlobalArgs {
    double* WW;         // N x N = W W^T (destroyed)
    int32_t N, K;
    int32_t max_sweeps;
    double* T;          // N x K: X~ diag(1 / Lambda~)
    double* Lam;        // K
    double* X;          // N x K
    double* vec;        // 2N
    int32_t* ivec;      // 3N
    int32_t* status;
    int32_t* sweeps;
};

// The paper's low-rank SVD of a small matrix (k_low_rank_small): Eqs. (7)-(11)
// without power iterations, one work-group.
struct LowRankArgs {
    int32_t m, n, l, K;        // A is m x n; test matrix n x l; k = min(K, l) triplets kept
    const double* A;           // element (i, j) at A[i * a_i + j * a_j]
    int64_t a_i, a_j;
    const double* Om;          // n x l, column-major (ld n)
    int32_t max_sweeps;
    double* work;              // low_rank_work_doubles(m, n, l)
    double* U;                 // m x k out (ld ldu): the left singular vectors Q U~_k
    int64_t ldu;
    double* s;                 // k out
    int32_t post;              // 0: none; 1: T = R^-1 U with R = post_R (m x m upper, ld m);
                               // 2: T = U diag(1 / s) with the small-value check
    const double* post_R;
    double* T;                 // m x k out (ld m) for post 1 and 2
    int32_t* status;
    int32_t* sweeps;
};
size_t low_rank_work_doubles(int m, int n, int l);

struct GradCoreArgs {
    int32_t n, r, rk;
    const double* R;      // n x n upper Cholesky-QR factor of the panel
    const double* Ut;     // n x n left singular vectors of R (sorted, sign rule)
    const double* S;      // n singular values
    const double* E;      // n x rk: C^T U_bar (C with its column scale)
    const double* sbar;   // rk
    const double* d;      // r column scale of the U part (ff * s_prev)
    double* Tf;           // n x n work
    double* V;            // n x n work
    double* H;            // n x rk work
    double* Wk;           // n x n work
    double* Zt;           // n x n work
    double* Zu;           // (n + rk) x r out (ld n + rk)
    double* Za;           // (n + rk) x (n - r) out (ld n + rk)
    int32_t* status;
};

hipError_t launch_grad_core(const GradCoreArgs& a, hipStream_t st);
hipError_t launch_grad_sbar(const double* G, int r, const double* s_prev, double* sbar, hipStream_t st);

hipError_t launch_tn(bool fp64, const TnArgs& a, int nitems, hipStream_t st);
// launch_nn takes k_nn_x (one read of the panel, all output columns per
// work-group) for FP32 products on float4-aligned FP32 panels with 32 < nx <= 128.
inline bool nn_wide(bool fp64, const NnArgs& a) {
    return !fp64 && a.all_f32 && a.vec_f32 && a.n >= 1 && a.nx > 32 && a.nx <= 128;
}
// k_tn_x: non-symmetric FP32 P = L^T R on float4-aligned FP32 operands, R at
// most TNX_RCOLS columns; one work-group per (TNX_LCOLS columns of L, slot),
// slot s covering rows [s chunk, (s + 1) chunk) (chunk a multiple of 64).
constexpr int TNX_LCOLS = 320, TNX_RCOLS = 128;
hipError_t launch_tn_x(const TnArgs& a, int nslots, hipStream_t st);
hipError_t launch_tn_reduce(const TnReduceArgs& a, int nseg, hipStream_t st);
hipError_t launch_nn(bool fp64, const NnArgs& a, int nitems, hipStream_t st);
// Compiled configuration of a fused pass: tile height, padded panel width
// (the layout of the partial sums) and dynamic LDS bytes.
struct FusedPlan {
    int tm;
    int np;
    size_t lds;
};
// BF16 power pass (k_sketch_bf16) / FP32 passes (k_fused) for an n-column
// panel; tile_rows = 0 picks the default height.  false: no compiled kernel.
bool sketch_plan(int n, int tile_rows, FusedPlan* p);
bool fused_plan(int n, int tile_rows, FusedPlan* p, bool lift = false);
hipError_t launch_sketch_bf16(const FusedArgs& a, hipStream_t st);
// Final pass of the mixed precision with split-BF16 products (one column block).
bool split_plan(int n, FusedPlan* p);
hipError_t launch_final_split(const FusedArgs& a, hipStream_t st);
hipError_t launch_fused(int mode, const FusedArgs& a, hipStream_t st);   // FP32: 0 power, 1 final, 2 lift
// Final pass of the mixed precision with split-BF16 operands (k_split64) on
// float4-aligned panels, one column block: P = C^T (C X) and the kept Y
// (a.yout, a BF16 pair per value).
bool split64_plan(int n, FusedPlan* p);
hipError_t launch_split64(const FusedArgs& a, hipStream_t st);
// Fused pass with every operand split into `terms` BF16 terms (k_splitpass),
// float4-aligned panels, one column block, 32-row tiles; launched with
// terms = 3: an FP32-accurate power pass (P only, a.yout null).
bool splitpass_plan(int n, int terms, FusedPlan* p);
hipError_t launch_splitpass(int terms, const FusedArgs& a, hipStream_t st);
// G = Y^T Y of the kept sketch into nwg FP64 64 x 64 partials (k_gram_kept).
hipError_t launch_gram_kept(const float* Y, int64_t rows, int64_t ldy, int lx, int nwg, double* part, hipStream_t st);
hipError_t launch_fused_reduce(const FusedReduceArgs& a, hipStream_t st);

hipError_t launch_small_det1(const SmallArgs& a, hipStream_t st);
hipError_t launch_small_det2(const SmallArgs& a, hipStream_t st);
hipError_t launch_small_orth(const OrthArgs& a, hipStream_t st);
hipError_t launch_status_fold(int32_t* st, hipStream_t stream);
hipError_t launch_small_rand_final(const RandFinalArgs& a, hipStream_t st);
hipError_t launch_scale_rows(double* X, int n, int m, int ldx, const double* d, int r, int times, hipStream_t st);
// status (may be null): the status words are cleared in the same launch
hipError_t launch_make_scale(int32_t* status, double* d, const double* s, int r, double ff, hipStream_t st);
hipError_t launch_rand_begin(int32_t* status, double* d, const double* s, int r, double ff, double* X,
                             const double* Om, int n, int l, hipStream_t st);
hipError_t launch_apmos_local(const ApmosLocalArgs& a, hipStream_t st);
hipError_t launch_low_rank_small(const LowRankArgs& a, hipStream_t st);
hipError_t launch_apmos_global(const ApmosGlobalArgs& a, hipStream_t st);

}  // namespace psvd
