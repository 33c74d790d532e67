// small.hip -- FP64 small-core kernels, one work-group each.
//
// The tall passes reduce each update to matrices of size at most
// (r + N) x (r + N) or (K + p) x (K + p); these kernels factor them on the
// device so an update never waits for the host:
//   Cholesky R^T R = G with breakdown / non-finite detection,
//   triangular inverse, small products,
//   one-sided Jacobi SVD (Hestenes) with a parallel round-robin ordering,
//   stable descending sort, sign rule, truncation to K.
// All matrices are column-major FP64 in device memory (L2 resident).
#include "kernels.h"

namespace psvd {

constexpr int SM_THREADS = 1024;
constexpr int SM_WAVES = SM_THREADS / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ bool finite_d(double x) { return isfinite(x); }

// ---------------------------------------------------------------------------
// Cholesky, in place on the upper triangle: A = R^T R, R upper.
// Right-looking with one barrier per column: step k updates the trailing
// block (a_ij -= a_ki a_kj / a_kk, k < i <= j) from the still unscaled row k,
// and scales row k - 1 (which no thread reads in that step).  Threads form a
// 32 x (blockDim / 32) grid over (i, j).  Returns false (uniformly) on a
// non-positive or non-finite pivot; A is then partially overwritten.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool wg_chol_upper(double* A, int n, int lda) {
    const int tid = threadIdx.x;
    const int ti = tid & 31, tj = tid >> 5, TJ = blockDim.x >> 5;
    double d_prev = 1.0;
    for (int k = 0; k < n; ++k) {
        const double d = A[k + (size_t)k * lda];
        if (!(d > 0.0) || !finite_d(d)) {
            __syncthreads();
            return false;
        }
        if (k > 0 && tid < n - k + 1) {   // scale row k - 1 (one wave for n <= 64)
            const double rp = sqrt(d_prev), ip = 1.0 / rp;
            const int j = k - 1 + tid;
            A[(k - 1) + (size_t)j * lda] = (j == k - 1) ? rp : A[(k - 1) + (size_t)j * lda] * ip;
            for (int jj = j + blockDim.x; jj < n; jj += blockDim.x) A[(k - 1) + (size_t)jj * lda] *= ip;
        }
        if (tj < n - k - 1) {             // only threads with trailing work take the reciprocal
            const double invd = 1.0 / d;
            for (int j = k + 1 + tj; j < n; j += TJ) {
                const double akj = A[k + (size_t)j * lda] * invd;
                for (int i = k + 1 + ti; i <= j; i += 32) A[i + (size_t)j * lda] -= A[k + (size_t)i * lda] * akj;
            }
        }
        __syncthreads();
        d_prev = d;
    }
    if (tid == 0 && n > 0) A[(n - 1) + (size_t)(n - 1) * lda] = sqrt(d_prev);
    for (int j = tj; j < n; j += TJ)
        for (int i = j + 1 + ti; i < n; i += 32) A[i + (size_t)j * lda] = 0.0;
    __syncthreads();
    return true;
}

// Leading dimension of the LDS copy of the n <= 64 Cholesky (odd: a row
// spreads over the banks).
constexpr int CHOL64_LD = 65;

// Cholesky for n <= 64, blocked by 16: all threads call it, out = R with
// G + shift I = R^T R (G read from src, n x n, leading dimension n; out may be
// src; S: 64 x 65 doubles of LDS); false, uniformly, on a non-positive or
// non-finite pivot.
// The matrix is padded to 16 NB rows and columns with the identity.  Per
// diagonal block b:
//   1. wave 0 factors the 16 x 16 diagonal block in registers (lane j < 16
//      holds column 16b + j; the pivot and row of each step come by readlane);
//   2. R_12 = R_11^-T A_12 for the columns to its right, one lane per column
//      (forward substitution, R_11 read from LDS by every lane at once);
//   3. A_22 -= R_12^T R_12 on the FP64 matrix cores, upper 16 x 16 blocks over
//      the waves.
// Three barriers per block instead of one per column.
__device__ __forceinline__ double readlane_d(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// 1 / sqrt(x) for x > 0: the hardware estimate and two Newton steps (relative
// error a few units of 2^-53; not the correctly rounded value)
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x * y, y, 1.0);   // 1 - x y^2
        y = fma(0.5 * y, e, y);
    }
    return y;
}

__device__ __forceinline__ bool wg_chol64b(const double* src, int n, double shift, double* S, double* out) {
    constexpr int ld = CHOL64_LD;
    __shared__ int chol_ok;
    __shared__ double chol_rinv[64];   // 1 / R_kk
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
    const int NB = (n + 15) >> 4, np = NB * 16;
    for (int e = tid; e < np * np; e += blockDim.x) {
        const int i = e % np, j = e / np;
        S[i + j * ld] = (i < n && j < n) ? src[i + j * n] + (i == j ? shift : 0.0) : (i == j ? 1.0 : 0.0);
    }
    if (tid == 0) chol_ok = 1;
    __syncthreads();
    for (int b = 0; b < NB; ++b) {
        const int c0 = 16 * b;
        if (w == 0) {
            // 1. diagonal block: lane j < 16 holds column c0 + j, rows c0 .. c0 + 15
            double a[16];
            const int jc = c0 + (lane & 15);
#pragma unroll
            for (int i = 0; i < 16; ++i) a[i] = S[c0 + i + jc * ld];
            bool ok = true;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const double d = readlane_d(a[k], k);
                ok = ok && d > 0.0 && isfinite(d);
                const double ir = rsqrt_nr(d > 0.0 ? d : 1.0);
                // row k of R: lane k takes sqrt(d) = d / sqrt(d), the others scale.
                // Lanes j < k change only entries below the diagonal of their
                // finished columns, and lanes j < i below-diagonal entries of
                // theirs: no step reads those, so every lane runs every update.
                a[k] = (lane & 15) == k ? d * ir : a[k] * ir;
                if (lane == k) chol_rinv[c0 + k] = ir;
#pragma unroll
                for (int i = k + 1; i < 16; ++i) a[i] = fma(-readlane_d(a[k], i), a[k], a[i]);   // R[k][c0 + i]
            }
            if (lane < 16)
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    if (i <= lane) S[c0 + i + jc * ld] = a[i];
            if (lane == 0 && !ok) chol_ok = 0;
        }
        __syncthreads();
        if (c0 + 16 < np) {
            // 2. R_12: column c (right of the block) solves R_11^T x = a_c
            for (int c = c0 + 16 + tid; c < np; c += blockDim.x) {
                double x[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) x[i] = S[c0 + i + c * ld];
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    double s = x[i];
#pragma unroll
                    for (int m = 0; m < i; ++m) s = fma(-S[c0 + m + (c0 + i) * ld], x[m], s);
                    x[i] = s * chol_rinv[c0 + i];
                }
#pragma unroll
                for (int i = 0; i < 16; ++i) S[c0 + i + c * ld] = x[i];
            }
            __syncthreads();
            // 3. A_22 -= R_12^T R_12: upper 16 x 16 blocks (p <= q) of the trailing matrix
            const int mb = NB - b - 1;
            const int nblk = mb * (mb + 1) / 2;
            for (int t = w; t < nblk; t += nw) {
                int p = 0, q = t;
                while (q >= mb - p) { q -= mb - p; ++p; }
                q += p;                                     // p <= q < mb
                const int cp = c0 + 16 + 16 * p, cq = c0 + 16 + 16 * q;
                d4_t acc = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k4 = 0; k4 < 16; k4 += 4) {
                    const int kk = c0 + k4 + (lane >> 4);
                    const double av = S[kk + (cp + (lane & 15)) * ld];   // R_12^T (i, k) = R_12 (k, i)
                    const double bv = S[kk + (cq + (lane & 15)) * ld];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = cp + (lane >> 4) + 4 * v, col = cq + (lane & 15);
                    S[row + col * ld] -= acc[v];
                }
            }
            __syncthreads();
        }
    }
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e % n, j = e / n;
        out[e] = i <= j ? S[i + j * ld] : 0.0;
    }
    const bool ok = chol_ok != 0;
    __syncthreads();
    return ok;
}

// X (n x nrhs) = R^-1 B for upper triangular R (n x n), row by row from the
// bottom: step i fixes row i of X for every right-hand side in parallel, so no
// thread ever waits on a value it has just stored.  B == nullptr means B = I
// (X = R^-1, upper triangular).  X must not alias R or B.
__device__ __forceinline__ void wg_trsm_upper(const double* R, int ldr, int n, const double* B, int ldb, double* X, int ldx,
                              int nrhs) {
    const int tid = threadIdx.x;
    for (int i = n - 1; i >= 0; --i) {
        const double rii = R[i + (size_t)i * ldr];
        for (int j = tid; j < nrhs; j += blockDim.x) {
            double s;
            int kend = n;
            if (B) {
                s = B[i + (size_t)j * ldb];
            } else {
                s = (i == j) ? 1.0 : 0.0;
                kend = j + 1;                       // rows k > j of column j of R^-1 are zero
                if (i > j) {
                    X[i + (size_t)j * ldx] = 0.0;
                    continue;
                }
            }
            for (int k = i + 1; k < kend; ++k) s -= R[i + (size_t)k * ldr] * X[k + (size_t)j * ldx];
            X[i + (size_t)j * ldx] = s / rii;
        }
        __syncthreads();
    }
}

// Sum over the 16 lanes of a row (quarter-wave) by DPP row rotations (8, 4,
// 2, 1): every lane ends with the same value (each step adds the same two
// partial sums on both lanes of a pair).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double q16_sum(double v) {
    v += dpp_d<0x128>(v);   // row_ror:8
    v += dpp_d<0x124>(v);   // row_ror:4
    v += dpp_d<0x122>(v);   // row_ror:2
    v += dpp_d<0x121>(v);   // row_ror:1
    return v;
}

// Ri = R^-1 for upper triangular R (n x n); one quarter-wave per column j
// runs the back substitution R x = e_j (rows j .. 0), the partial sums of
// each row split over its 16 lanes.  Every lane stores the (identical) x_i,
// so each later read is of a value the reading lane wrote itself.
// rinv: n doubles of scratch.  R, Ri, rinv distinct.
__device__ __forceinline__ void wg_trinv_upper(const double* R, int n, int ldr, double* Ri, int ldi, double* rinv) {
    const int tid = threadIdx.x, ql = tid & 15, qw = tid >> 4, nq = blockDim.x >> 4;
    for (int i = tid; i < n; i += blockDim.x) rinv[i] = 1.0 / R[i + (size_t)i * ldr];
    __syncthreads();
    for (int j = qw; j < n; j += nq) {
        double* x = Ri + (size_t)j * ldi;
        for (int i = j + 1 + ql; i < n; i += 16) x[i] = 0.0;
        for (int i = j; i >= 0; --i) {
            double s = 0.0;
            for (int k = i + 1 + ql; k <= j; k += 16) s += R[i + (size_t)k * ldr] * x[k];
            s = q16_sum(s);
            x[i] = ((i == j ? 1.0 : 0.0) - s) * rinv[i];
        }
    }
    __syncthreads();
}

// C = op(A) B over one work-group on the FP64 16x16x4 matrix cores.
// op(A)(i, k) = A[i * a_i + k * a_k];  B(k, j) = B[k * b_k + j * b_j];
// C(i, j) -> C[i * c_i + j * c_j], multiplied by rs[i] for i < nrs when rs is
// given.  16 x 16 output tiles are dealt to the waves round-robin; the sum
// over k runs in a fixed order (two interleaved accumulators, added last).
// Operands may live in LDS or global memory; C must not alias them.
__device__ __forceinline__ void wg_gemm_f64(int m, int n, int k, const double* A, int a_i, int a_k, const double* B,
                                         int b_k, int b_j, double* C, int c_i, int c_j, const double* rs, int nrs) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int mt = (m + 15) >> 4, nt = (n + 15) >> 4;
    const int kl = lane >> 4;
    for (int t = w; t < mt * nt; t += nw) {
        const int ib = t % mt, jb = t / mt;
        const int i = ib * 16 + (lane & 15), j = jb * 16 + (lane & 15);
        const int ic = i < m ? i : m - 1, jc = j < n ? j : n - 1;
        d4_t acc0 = d4_t{0.0, 0.0, 0.0, 0.0}, acc1 = d4_t{0.0, 0.0, 0.0, 0.0};
        // KU k-steps of 4 per batch: all their loads are issued before the matrix-core work
        constexpr int KU = 16;
        for (int k0 = 0; k0 < k; k0 += 4 * KU) {
            double av[KU], bv[KU];
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int kk = k0 + 4 * u + kl;
                const int kc = kk < k ? kk : k - 1;
                av[u] = A[(size_t)ic * a_i + (size_t)kc * a_k];
                bv[u] = B[(size_t)kc * b_k + (size_t)jc * b_j];
            }
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const int kk = k0 + 4 * u + kl;
                const double a0 = (i < m && kk < k) ? av[u] : 0.0;
                const double b0 = (j < n && kk < k) ? bv[u] : 0.0;
                if (u & 1) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc1, 0, 0, 0);
                else acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc0, 0, 0, 0);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = ib * 16 + kl + 4 * v, col = jb * 16 + (lane & 15);
            if (row < m && col < n) {
                double x = acc0[v] + acc1[v];
                if (rs && row < nrs) x *= rs[row];
                C[(size_t)row * c_i + (size_t)col * c_j] = x;
            }
        }
    }
    __syncthreads();
}

// C (m x n) = A (m x k) * B (k x n); all column-major, parallel over outputs.
__device__ void wg_gemm_nn(int m, int n, int k, const double* A, int lda, const double* B, int ldb, double* C,
                           int ldc) {
    for (int e = threadIdx.x; e < m * n; e += SM_THREADS) {
        int i = e % m, j = e / m;
        double s = 0.0;
        for (int p = 0; p < k; ++p) s += A[i + (size_t)p * lda] * B[p + (size_t)j * ldb];
        C[i + (size_t)j * ldc] = s;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Products with a tall operand P (n x l, column-major, ld ldp, l <= 64) in
// global memory, staged through LDS in coalesced chunks of 64 rows
// (Cn: 64 x 65 doubles, column-major); the next chunk is prefetched into
// registers while the matrix cores work on the current one.
// ---------------------------------------------------------------------------
constexpr int TALL_KC = 64;
constexpr int TALL_LDC = 65;
constexpr int TALL_CHUNK = TALL_KC * TALL_LDC;   // doubles of the LDS chunk
static_assert(TALL_CHUNK >= 64 * CHOL64_LD, "the chunk also holds the n <= 64 Cholesky copy");

struct TallStager {
    // Loads only (at clamped, always valid addresses): nothing reads the
    // loaded values before `store`, so the loads of the next chunk stay in
    // flight while the matrix cores work on the current one; the mask of rows
    // past n and columns past l is applied at the store.
    double pre[4];
    __device__ __forceinline__ void fetch(const double* P, int n, int l, int ldp, int r0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + q * blockDim.x;
            const int r = e & 63, c = e >> 6;
            const int rc = r0 + r < n ? r0 + r : n - 1, cc = c < l ? c : l - 1;
            pre[q] = gldd(P + rc + (size_t)cc * ldp);
        }
    }
    __device__ __forceinline__ void store(double* Cn, int n, int l, int r0) {
        const int lp = ((l + 15) >> 4) << 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + q * blockDim.x;
            const int r = e & 63, c = e >> 6;
            if (e < TALL_KC * lp) Cn[c * TALL_LDC + r] = (c < l && r0 + r < n) ? pre[q] : 0.0;
        }
    }
};

// G (l x l, ld ldg; may be in LDS) = P^T P.  Upper 16 x 16 tiles, one per
// wave, mirrored on output.  blockDim.x >= 640 (10 tiles for l <= 64).
__device__ __forceinline__ void wg_gram_tall(int n, int l, const double* P, int ldp, double* G, int ldg, double* Cn) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int mt = (l + 15) >> 4;
    const int ntile = mt * (mt + 1) / 2;
    int t = w, jb = 0;
    while (t > jb) {
        t -= jb + 1;
        ++jb;
    }
    const int ib = t;
    const bool has = w < ntile;
    d4_t acc0 = d4_t{0.0, 0.0, 0.0, 0.0}, acc1 = d4_t{0.0, 0.0, 0.0, 0.0};
    TallStager st;
    st.fetch(P, n, l, ldp, 0);
    for (int k0 = 0; k0 < n; k0 += TALL_KC) {
        st.store(Cn, n, l, k0);
        lds_barrier();   // waves exchange only the LDS chunk: the prefetch stays in flight
        if (k0 + TALL_KC < n) st.fetch(P, n, l, ldp, k0 + TALL_KC);
        if (has) {
            const double* ca = Cn + (ib * 16 + (lane & 15)) * TALL_LDC + (lane >> 4);
            const double* cb = Cn + (jb * 16 + (lane & 15)) * TALL_LDC + (lane >> 4);
#pragma unroll
            for (int kk = 0; kk < TALL_KC; kk += 8) {
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[kk], cb[kk], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[kk + 4], cb[kk + 4], acc1, 0, 0, 0);
            }
        }
        lds_barrier();
    }
    if (has) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = ib * 16 + (lane >> 4) + 4 * v, col = jb * 16 + (lane & 15);
            if (row < l && col < l) {
                const double x = acc0[v] + acc1[v];
                G[row + (size_t)col * ldg] = x;
                G[col + (size_t)row * ldg] = x;
            }
        }
    }
    __syncthreads();
}

// X (n x l, ld ldx, global) = diag(rs) P B with B (l x l, ld ldb) and rows
// i < nrs scaled by rs[i] (rs may be null).  Wave w: rows 16 (w & 3) of the
// chunk, columns 16 (w >> 2).  blockDim.x == 1024.
__device__ __forceinline__ void wg_mul_tall(int n, int l, const double* P, int ldp, const double* B, int ldb, double* X,
                                         int ldx, const double* rs, int nrs, double* Cn) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int mt = (l + 15) >> 4;
    const int rb = w & 3, cb = w >> 2;
    const bool has = cb < mt;
    // B fragments of this wave's column block, all k-steps (<= 16)
    double bf[16];
    {
        const int j = cb * 16 + (lane & 15);
        const int jc = j < l ? j : l - 1;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int k = 4 * u + (lane >> 4);
            const int kc = k < l ? k : l - 1;
            const double v = B[kc + (size_t)jc * ldb];
            bf[u] = (has && j < l && k < l) ? v : 0.0;
        }
    }
    TallStager st;
    st.fetch(P, n, l, ldp, 0);
    for (int r0 = 0; r0 < n; r0 += TALL_KC) {
        st.store(Cn, n, l, r0);
        lds_barrier();
        if (r0 + TALL_KC < n) st.fetch(P, n, l, ldp, r0 + TALL_KC);
        if (has) {
            d4_t acc0 = d4_t{0.0, 0.0, 0.0, 0.0}, acc1 = d4_t{0.0, 0.0, 0.0, 0.0};
            const double* ca = Cn + (lane >> 4) * TALL_LDC + rb * 16 + (lane & 15);
#pragma unroll
            for (int u = 0; u < 16; u += 2) {
                if (4 * u < l) acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[(4 * u) * TALL_LDC], bf[u], acc0, 0, 0, 0);
                if (4 * u + 4 < l)
                    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[(4 * u + 4) * TALL_LDC], bf[u + 1], acc1, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = r0 + rb * 16 + (lane >> 4) + 4 * v, col = cb * 16 + (lane & 15);
                if (row < n && col < l) {
                    double x = acc0[v] + acc1[v];
                    if (rs && row < nrs) x *= rs[row];
                    X[row + (size_t)col * ldx] = x;
                }
            }
        }
        lds_barrier();
    }
    __syncthreads();   // X complete before the caller reads it
}

// One Jacobi pair (columns zp, zq of m rows, squared norms al, be) by one
// quarter-wave: the inner product, the tests and, unless the pair is already
// orthogonal to tol or a column is negligible, the rotation with |angle| <=
// pi/4 that makes the columns orthogonal:
//   u = |be - al| + sqrt((be - al)^2 + 4 g^2),  h = 1 / sqrt(u^2 + 4 g^2),
//   c = u h,  s = sign(be - al) 2 g h   (tan = s / c),
// and the squared norms of the rotated columns (lane 0 of the group).
// jac_pair_regs holds columns of at most 16 E rows in registers (E entries
// per lane, clamped reads masked to zero); jac_pair_loop takes any m.
__device__ __forceinline__ void jac_rotate_norms(double c, double s, double g, double al, double be, double* np,
                                                 double* nq, int* sflag) {
    const double cs2g = 2.0 * c * s * g;
    *np = c * c * al + s * s * be - cs2g;
    *nq = s * s * al + c * c * be + cs2g;
    *sflag = 1;
}

__device__ __forceinline__ bool jac_angle(double g, double al, double be, double negl, double tol, double* c,
                                          double* s) {
    if (!(al > negl) || !(be > negl)) return false;
    if (g * g <= (tol * tol) * (al * be)) return false;   // |g| <= tol sqrt(al be)
    const double dif = be - al;
    // the hardware square root sets the angle only; c and s share one
    // correctly rounded reciprocal square root, so the rotation stays
    // orthogonal to rounding
    const double uu = fabs(dif) + __builtin_amdgcn_sqrt(dif * dif + 4.0 * g * g);
    const double hh = rsqrt(uu * uu + 4.0 * g * g);
    *c = uu * hh;
    *s = (dif >= 0.0 ? 2.0 * g : -2.0 * g) * hh;
    return true;
}

template <int E>
__device__ __forceinline__ void jac_pair_regs(double* zp, double* zq, int m, int ql, double al, double be, double negl,
                                              double tol, double* np, double* nq, int* sflag, double stop, int* sfar) {
    double xp[E], xq[E];
    double g = 0.0;
#pragma unroll
    for (int u = 0; u < E; ++u) {
        const int i = ql + 16 * u;
        const int ic = i < m ? i : m - 1;
        xp[u] = zp[ic];
        xq[u] = zq[ic];
        if (i >= m) xp[u] = xq[u] = 0.0;
        g += xp[u] * xq[u];
    }
    g = q16_sum(g);
    if (stop > 0.0 && ql == 0 && al > negl && be > negl && g * g > stop * (al * be)) *sfar = 1;
    double c, s;
    if (!jac_angle(g, al, be, negl, tol, &c, &s)) return;
#pragma unroll
    for (int u = 0; u < E; ++u) {
        const int i = ql + 16 * u;
        if (i < m) {
            zp[i] = c * xp[u] - s * xq[u];
            zq[i] = s * xp[u] + c * xq[u];
        }
    }
    if (ql == 0) jac_rotate_norms(c, s, g, al, be, np, nq, sflag);
}

// jac_pair_regs with 16-byte accesses: lane ql holds rows 32 u + 2 ql and the
// next (u < E2, at most 32 E2 rows); m even and the columns 16-byte aligned.
template <int E2>
__device__ __forceinline__ void jac_pair_regs2(double* zp, double* zq, int m, int ql, double al, double be, double negl,
                                               double tol, double* np, double* nq, int* sflag, double stop, int* sfar) {
    double xp[2 * E2], xq[2 * E2];
    double g = 0.0;
#pragma unroll
    for (int u = 0; u < E2; ++u) {
        const int i = 32 * u + 2 * ql;
        const int ic = i < m ? i : m - 2;
        d2_t a = *(const d2_t*)(zp + ic), b = *(const d2_t*)(zq + ic);
        if (i >= m) a = b = d2_t{0.0, 0.0};
        xp[2 * u] = a[0];
        xp[2 * u + 1] = a[1];
        xq[2 * u] = b[0];
        xq[2 * u + 1] = b[1];
        g = fma(a[0], b[0], g);
        g = fma(a[1], b[1], g);
    }
    g = q16_sum(g);
    if (stop > 0.0 && ql == 0 && al > negl && be > negl && g * g > stop * (al * be)) *sfar = 1;
    double c, s;
    if (!jac_angle(g, al, be, negl, tol, &c, &s)) return;
#pragma unroll
    for (int u = 0; u < E2; ++u) {
        const int i = 32 * u + 2 * ql;
        if (i < m) {
            *(d2_t*)(zp + i) = d2_t{c * xp[2 * u] - s * xq[2 * u], c * xp[2 * u + 1] - s * xq[2 * u + 1]};
            *(d2_t*)(zq + i) = d2_t{s * xp[2 * u] + c * xq[2 * u], s * xp[2 * u + 1] + c * xq[2 * u + 1]};
        }
    }
    if (ql == 0) jac_rotate_norms(c, s, g, al, be, np, nq, sflag);
}

__device__ __forceinline__ void jac_pair_loop(double* zp, double* zq, int m, int ql, double al, double be, double negl,
                                              double tol, double* np, double* nq, int* sflag, double stop, int* sfar) {
    double g = 0.0;
    for (int i = ql; i < m; i += 16) g += zp[i] * zq[i];
    g = q16_sum(g);
    if (stop > 0.0 && ql == 0 && al > negl && be > negl && g * g > stop * (al * be)) *sfar = 1;
    double c, s;
    if (!jac_angle(g, al, be, negl, tol, &c, &s)) return;
    for (int i = ql; i < m; i += 16) {
        const double a = zp[i], b = zq[i];
        zp[i] = c * a - s * b;
        zq[i] = s * a + c * b;
    }
    if (ql == 0) jac_rotate_norms(c, s, g, al, be, np, nq, sflag);
}

// ---------------------------------------------------------------------------
// One-sided Jacobi on the columns of Z (m x n, ldz), in place.  On return
// the columns are mutually orthogonal to the tolerance m * 2^-53; sig[j] =
// ||z_j|| and z_j /= sig[j] (0 columns stay 0).  order[0..n) lists the
// columns by descending sig (stable).  Parallel round-robin ordering: each
// round rotates n/2 disjoint pairs, one pair per quarter-wave (16 lanes) at a time.
// With cmap, column j of the iteration is column cmap[j] of Z (sig, order and
// nrm stay indexed by j).  acc16 asks for 16-byte accesses (two rows per lane
// and access; taken when m and ldz are even and Z is 16-byte aligned): faster
// for the 120 x 120 matrix of the wide randomized core, slower for the 74-row
// R and the 128-row APMOS factors, so callers choose.  stop_cos2 > 0 ends the
// iteration after a sweep whose largest squared cosine g^2 / (al be) is at most
// max(stop_cos2, tol), as wg_jacobi_pad64 does (convergence is quadratic).
// Returns the number of sweeps (> max_sweeps: not converged).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wg_jacobi(double* Z, int m, int n, int ldz, double* sig, int* order, double* nrm,
                                         int max_sweeps, int* sflag, const int* cmap = nullptr, bool acc16 = false,
                                         double stop_cos2 = 0.0) {
    __shared__ int jfar;   // a pair of this sweep had cos^2 above the early-end bound
    // One pair per quarter-wave (16 lanes): a round of n/2 disjoint pairs runs
    // in one pass when blockDim.x / 16 >= n / 2.
    const int tid = threadIdx.x;
    const int ql = tid & 15, qw = tid >> 4, nq = blockDim.x >> 4;
    const double tol = (double)m * 0x1p-53;
    const int ne = n + (n & 1);
    const bool v2 = acc16 && (m % 2) == 0 && (ldz % 2) == 0 && ((uintptr_t)Z % 16) == 0;
    const double stop = stop_cos2 > 0.0 ? (stop_cos2 > tol ? stop_cos2 : tol) : 0.0;
    int sweep = 0;
    for (;;) {
        for (int j = qw; j < n; j += nq) {
            const double* z = Z + (size_t)(cmap ? cmap[j] : j) * ldz;
            double s = 0.0;
            for (int i = ql; i < m; i += 16) s += z[i] * z[i];
            s = q16_sum(s);
            if (ql == 0) nrm[j] = s;
        }
        if (tid == 0) {
            *sflag = 0;
            jfar = 0;
        }
        __syncthreads();
        if (tid < 64) {   // largest squared norm, by wave 0, broadcast through nrm[n]
            double mx = 0.0;
            for (int j = tid; j < n; j += 64) mx = fmax(mx, nrm[j]);
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
            if (tid == 0) nrm[n] = mx;
        }
        __syncthreads();
        const double negl = nrm[n] * tol * tol;
        if (sweep >= max_sweeps) {
            ++sweep;
            break;
        }
        for (int t = 0; t < ne - 1; ++t) {
            for (int pi = qw; pi < ne / 2; pi += nq) {
                const int pa = pi, pb = ne - 1 - pi;
                int xa = pa - 1 + t, xb = pb - 1 + t;   // (pa - 1 + t) mod (ne - 1), both < 2 (ne - 1)
                xa -= xa >= ne - 1 ? ne - 1 : 0;
                xb -= xb >= ne - 1 ? ne - 1 : 0;
                const int ca = pa == 0 ? 0 : 1 + xa;
                const int cb = pb == 0 ? 0 : 1 + xb;
                const int p = ca < cb ? ca : cb, q = ca < cb ? cb : ca;
                if (q >= n) continue;
                double* zp = Z + (size_t)(cmap ? cmap[p] : p) * ldz;
                double* zq = Z + (size_t)(cmap ? cmap[q] : q) * ldz;
                const double al = nrm[p], be = nrm[q];
                // entries per lane: the fewest that hold m rows (pairs of rows per
                // 16-byte access when m and the leading dimension are even)
                if (v2 && m <= 32) jac_pair_regs2<1>(zp, zq, m, ql, al, be, negl, tol, nrm + p, nrm + q, sflag, stop, &jfar);
                else if (v2 && m <= 64) jac_pair_regs2<2>(zp, zq, m, ql, al, be, negl, tol, nrm + p, nrm + q, sflag, stop, &jfar);
                else if (v2 && m <= 96) jac_pair_regs2<3>(zp, zq, m, ql, al, be, negl, tol, nrm + p, nrm + q, sflag, stop, &jfar);
                else if (v2 && m <= 128) jac_pair_regs2<4>(zp, zq, m, ql, al, be, negl, tol, nrm + p, nrm + q, sflag, stop, &jfar);
                else if (m <= 64) jac_pair_regs<4>(zp, zq, m, ql, al, be, negl, tol, nrm + p, nrm + q, sflag, stop, &jfar);
                else if (m <= 80) jac_pair_regs<5>(zp, zq, m, ql, al, be, negl, tol, nrm + p, nrm + q, sflag, stop, &jfar);
                else if (m <= 96) jac_pair_regs<6>(zp, zq, m, ql, al, be, negl, tol, nrm + p, nrm + q, sflag, stop, &jfar);
                else if (m <= 112) jac_pair_regs<7>(zp, zq, m, ql, al, be, negl, tol, nrm + p, nrm + q, sflag, stop, &jfar);
                else if (m <= 128) jac_pair_regs<8>(zp, zq, m, ql, al, be, negl, tol, nrm + p, nrm + q, sflag, stop, &jfar);
                else jac_pair_loop(zp, zq, m, ql, al, be, negl, tol, nrm + p, nrm + q, sflag, stop, &jfar);
            }
            __syncthreads();
        }
        ++sweep;
        const int rotated = *sflag, far = jfar;
        __syncthreads();
        if (!rotated || (stop > 0.0 && !far)) break;
    }
    // singular values, normalisation
    for (int j = qw; j < n; j += nq) {
        double* z = Z + (size_t)(cmap ? cmap[j] : j) * ldz;
        double s = 0.0;
        for (int i = ql; i < m; i += 16) s += z[i] * z[i];
        s = sqrt(q16_sum(s));
        for (int i = ql; i < m; i += 16) z[i] = s > 0.0 ? z[i] / s : 0.0;
        if (ql == 0) sig[j] = s;
    }
    __syncthreads();
    // stable descending order
    for (int j = tid; j < n; j += blockDim.x) {
        const double sj = sig[j];
        int rank = 0;
        for (int i = 0; i < n; ++i) {
            const double si = sig[i];
            if (si > sj || (si == sj && i < j)) ++rank;
        }
        order[rank] = j;
    }
    __syncthreads();
    return sweep;
}

// One-sided Jacobi for at most 64 rows and 64 columns, Z in LDS with leading
// dimension 64 and rows m..63 zero: every load and store of a pair is
// unconditional and the column norms are read before the dot product.  The
// same round-robin pairs, tests and rotation as wg_jacobi (both take the
// hardware square root for the angle term), with one change: a sweep whose
// largest squared cosine g^2 / (al be) is at most max(stop_cos2, tol) ends
// the iteration: convergence is quadratic, so the next sweep would take the
// cosines to about the square of that bound (tol: the sweep after it would
// only confirm cosines near tol).
// mx: 65 doubles of scratch.  Returns the sweep count (> max_sweeps: not
// converged); results as wg_jacobi.
__device__ __forceinline__ int wg_jacobi_pad64(double* Z, int m, int n, double* sig, int* order, double* nrm,
                                               int max_sweeps, int* sflag, double* mx, double stop_cos2) {
    constexpr int ldz = 64;
    const int tid = threadIdx.x;
    const int ql = tid & 15, qw = tid >> 4, nq = blockDim.x >> 4;
    const double tol = (double)m * 0x1p-53;
    const double stop = stop_cos2 > tol ? stop_cos2 : tol;
    const int ne = n + (n & 1);
    // quarter-wave qw < ne / 2 holds round-robin positions qw and ne - 1 - qw
    const int pa = qw, pb = ne - 1 - qw;
    const bool has_pair = qw < ne / 2;
    int sweep = 0;
    for (;;) {
        for (int j = qw; j < n; j += nq) {
            const double* z = Z + j * ldz + ql;
            double s0 = z[0] * z[0], s1 = z[16] * z[16];
            s0 = fma(z[32], z[32], s0);
            s1 = fma(z[48], z[48], s1);
            const double s = q16_sum(s0 + s1);
            if (ql == 0) nrm[j] = s;
        }
        if (tid == 0) *sflag = 0;
        __syncthreads();
        if (tid < 64) {   // largest squared norm, broadcast through nrm[n]
            double v = 0.0;
            for (int j = tid; j < n; j += 64) v = fmax(v, nrm[j]);
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
            if (tid == 0) nrm[n] = v;
        }
        __syncthreads();
        const double negl = nrm[n] * tol * tol;
        if (sweep >= max_sweeps) {
            ++sweep;
            break;
        }
        bool far = false;   // a pair of this quarter-wave had g^2 > stop al be
        for (int t = 0; t < ne - 1; ++t) {
            if (has_pair) {
                int xa = pa - 1 + t, xb = pb - 1 + t;   // (pos - 1 + t) mod (ne - 1), both < 2 (ne - 1)
                xa -= xa >= ne - 1 ? ne - 1 : 0;
                xb -= xb >= ne - 1 ? ne - 1 : 0;
                const int ca = pa == 0 ? 0 : 1 + xa;
                const int cb = 1 + xb;                   // pb >= ne / 2 > 0
                const int p = ca < cb ? ca : cb, q = ca < cb ? cb : ca;
                if (q < n) {
                    // lane ql holds rows 2 ql, 2 ql + 1, 32 + 2 ql, 33 + 2 ql: two
                    // 16-byte accesses per column
                    double* zp = Z + p * ldz + 2 * ql;
                    double* zq = Z + q * ldz + 2 * ql;
                    const double al = nrm[p], be = nrm[q];
                    const d2_t p0 = *(const d2_t*)zp, p1 = *(const d2_t*)(zp + 32);
                    const d2_t q0 = *(const d2_t*)zq, q1 = *(const d2_t*)(zq + 32);
                    const double xp[4] = {p0[0], p0[1], p1[0], p1[1]};
                    const double xq[4] = {q0[0], q0[1], q1[0], q1[1]};
                    double g0 = xp[0] * xq[0], g1 = xp[1] * xq[1];
                    g0 = fma(xp[2], xq[2], g0);
                    g1 = fma(xp[3], xq[3], g1);
                    const double g = q16_sum(g0 + g1);
                    if (al > negl && be > negl) {
                        const double gg = g * g, ab = al * be;
                        far = far || gg > stop * ab;
                        if (gg > (tol * tol) * ab) {
                            const double dif = be - al;
                            const double uu = fabs(dif) + __builtin_amdgcn_sqrt(fma(dif, dif, 4.0 * gg));
                            const double hh = rsqrt(fma(uu, uu, 4.0 * gg));
                            const double c = uu * hh, s = (dif >= 0.0 ? 2.0 * g : -2.0 * g) * hh;
                            *(d2_t*)zp = d2_t{c * xp[0] - s * xq[0], c * xp[1] - s * xq[1]};
                            *(d2_t*)(zp + 32) = d2_t{c * xp[2] - s * xq[2], c * xp[3] - s * xq[3]};
                            *(d2_t*)zq = d2_t{s * xp[0] + c * xq[0], s * xp[1] + c * xq[1]};
                            *(d2_t*)(zq + 32) = d2_t{s * xp[2] + c * xq[2], s * xp[3] + c * xq[3]};
                            if (ql == 0) {
                                const double cs2g = 2.0 * c * s * g;
                                nrm[p] = c * c * al + s * s * be - cs2g;
                                nrm[q] = s * s * al + c * c * be + cs2g;
                                *sflag = 1;
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (ql == 0 && qw < 64) mx[qw] = far ? 1.0 : 0.0;
        __syncthreads();
        if (tid < 64) {
            double v = tid < nq ? mx[tid] : 0.0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
            if (tid == 0) mx[64] = v;
        }
        ++sweep;
        __syncthreads();
        const bool done = !*sflag || mx[64] == 0.0;
        __syncthreads();
        if (done) break;
    }
    for (int j = qw; j < n; j += nq) {
        double* z = Z + j * ldz;
        double s = 0.0;
        for (int i = ql; i < m; i += 16) s += z[i] * z[i];
        s = sqrt(q16_sum(s));
        for (int i = ql; i < m; i += 16) z[i] = s > 0.0 ? z[i] / s : 0.0;
        if (ql == 0) sig[j] = s;
    }
    __syncthreads();
    for (int j = tid; j < n; j += blockDim.x) {
        const double sj = sig[j];
        int rank = 0;
        for (int i = 0; i < n; ++i) {
            const double si = sig[i];
            if (si > sj || (si == sj && i < j)) ++rank;
        }
        order[rank] = j;
    }
    __syncthreads();
    return sweep;
}

// Eigen-decomposition of a symmetric positive semi-definite matrix A (n x n,
// column-major with leading dimension n, both triangles stored), in place, by
// a rank-revealing Cholesky factorisation and one-sided Jacobi on the factor
// (the preconditioned one-sided Jacobi SVD of Drmac and Veselic, applied to
// the Cholesky factor of A instead of the R of a QR of the data):
//   1. Diagonal pivoting: step k takes the largest diagonal entry d of the
//      Schur complement (lowest index p on ties) and subtracts
//      A(:, p) A(:, p)^T / d from the rows and columns still in play; it stops
//      once d <= tolf max_j A_jj.  tolf = n 2^-53 is LAPACK's default tolerance
//      for its pivoted Cholesky (xPSTRF): the complement left out is within
//      the backward error of the factorisation.  For the Gram of FP32 data,
//      tolf = n 2^-48: the rounding E of the data (|E| <= 2^-24 |data|) has
//      ||E||^2 <= 2^-48 trace(A) <= n 2^-48 max_j A_jj, so eigenvalues below
//      that are the data's rounding.  Column p keeps its step-k entries: at the
//      rows still in play they are d^(1/2) times row k of the factor R, where
//      A ~ R^T R over the r pivots.
//   2. B = R^T (n x r, rows in the original index order, A ~ B B^T) is formed
//      in place in the pivot columns; every other column is cleared.
//   3. One-sided Jacobi on the r columns of B: B V = W with orthogonal
//      columns, A ~ W W^T, so the normalised columns of W are eigenvectors of
//      A with eigenvalues ||w_j||^2.  The pivoted factor's columns are graded
//      and there are r <= n of them: far fewer rounds than Jacobi on A.
// On return, for j in [0, n): column col[j] of A holds the unit eigenvector of
// the j-th largest eigenvalue sv[j]^2 (sv descending; the n - r columns past
// the rank are zero, with sv = 0).  Scratch: sig (n doubles), nrm (n + 1
// doubles, returned as sv), ord, state and cmap (n ints each; state is
// returned as col).  Returns the Jacobi sweep count (> max_sweeps: not
// converged).
__device__ int wg_psd_eig(double* A, int n, double* sig, double* nrm, int* ord, int* state, int* cmap,
                          int max_sweeps, int* sflag, double** sv, int** col, double tolf) {
    const int tid = threadIdx.x, lane = tid & 63, nt = blockDim.x;
    for (int j = tid; j < n; j += nt) state[j] = -1;   // state[j]: step at which j was pivoted
    double dm = 0.0;   // largest diagonal entry, by every wave alike
    for (int j = lane; j < n; j += 64) dm = fmax(dm, A[j + (size_t)j * n]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dm = fmax(dm, __shfl_xor(dm, off, 64));
    const double tol = dm * tolf;
    __syncthreads();
    int r = 0, prev = -1;
    for (; r < n; ++r) {
        // Every wave finds the same pivot from the same data.  The pivot of
        // the step before is excluded by register: thread 0 records it in
        // state[] during this step, while other waves may still be reading.
        double bv = -1.0;
        int bi = n;
        for (int j = lane; j < n; j += 64) {
            if (j == prev || state[j] >= 0) continue;
            const double v = A[j + (size_t)j * n];
            if (v > bv) {
                bv = v;
                bi = j;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (!(bv > tol)) break;
        const int p = bi;
        if (tid == 0) {
            if (prev >= 0) state[prev] = r - 1;
            cmap[r] = p;
        }
        const double inv = 1.0 / bv;
        const double* ap = A + (size_t)p * n;   // column p: not written in this step
        for (int j = tid >> 6; j < n; j += nt >> 6) {   // a wave per column still in play
            if (j == p || j == prev || state[j] >= 0) continue;
            const double fj = ap[j] * inv;
            double* aj = A + (size_t)j * n;
            for (int i = lane; i < n; i += 64)
                if (i != p && i != prev && state[i] < 0) aj[i] -= ap[i] * fj;
        }
        prev = p;
        __syncthreads();
    }
    if (tid == 0 && prev >= 0) state[prev] = r - 1;
    __syncthreads();
    for (int k = tid; k < r; k += nt) {   // the pivots d_k
        const int q = cmap[k];
        nrm[k] = A[q + (size_t)q * n];
    }
    for (int j = tid; j < n; j += nt) {   // indices never pivoted, ascending, after the pivots
        if (state[j] >= 0) continue;
        int c = 0;
        for (int i = 0; i < j; ++i) c += state[i] < 0;
        cmap[r + c] = j;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += nt) {   // B = R^T in the pivot columns
        const int i = e % n, j = e / n;
        const int kj = state[j], ki = state[i];
        double v = 0.0;
        if (kj >= 0 && (ki < 0 || ki >= kj)) v = A[e] / sqrt(nrm[kj]);
        A[e] = v;
    }
    __syncthreads();
    const int sw = wg_jacobi(A, n, r, n, sig, ord, nrm, max_sweeps, sflag, cmap);
    for (int j = tid; j < n; j += nt) {
        state[j] = j < r ? cmap[ord[j]] : cmap[j];
        nrm[j] = j < r ? sig[ord[j]] : 0.0;
    }
    __syncthreads();
    *sv = nrm;
    *col = state;
    return sw;
}

// Sign rule: column j of X (rows x k) gets its largest-magnitude entry
// (lowest index on ties) non-negative; flips recorded in flip[j].
__device__ __forceinline__ void wg_sign_rule(double* X, int rows, int k, int ldx, double* flip) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int j = w; j < k; j += SM_WAVES) {
        double* x = X + (size_t)j * ldx;
        double bv = -1.0;
        int bi = 0x7fffffff;
        for (int i = lane; i < rows; i += 64) {
            double a = fabs(x[i]);
            if (a > bv || (a == bv && i < bi)) {
                bv = a;
                bi = i;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            double ov = __shfl_xor(bv, off, 64);
            int oi = __shfl_xor(bi, off, 64);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        double f = (bi < rows && x[bi] < 0.0) ? -1.0 : 1.0;
        if (f < 0.0)
            for (int i = lane; i < rows; i += 64) x[i] = -x[i];
        if (lane == 0 && flip) flip[j] = f;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Workspace of the small core (device, FP64).
// ---------------------------------------------------------------------------

// Largest order whose n x n FP64 working matrix (plus 3 n scratch) fits in LDS.
constexpr int SM_LDS_MAX_N = 140;

// Two n x n working matrices when they fit (n <= 90), else one (n <= 140).
constexpr int SM_LDS_TWO_N = 90;

__host__ __device__ inline size_t small_lds_bytes(int n) {
    if (n <= SM_LDS_TWO_N) return (2 * (size_t)n * n + 4 * (size_t)n + 8) * sizeof(double);
    return n <= SM_LDS_MAX_N ? ((size_t)n * n + 4 * (size_t)n + 8) * sizeof(double) : 64;
}

// Start of the 3n-double vector scratch inside the LDS buffer.
__device__ __forceinline__ double* lds_vecs(double* lds, int n) {
    return lds + (n <= SM_LDS_TWO_N ? 2 : 1) * (size_t)n * n;
}

// Working copy of an n x n matrix: LDS when it fits, else the global buffer itself.
__device__ __forceinline__ double* stage_in(double* lds, double* g, int n, bool in_lds) {
    if (!in_lds) return g;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) lds[e] = g[e];
    __syncthreads();
    return lds;
}

__device__ __forceinline__ void stage_out(const double* w, double* g, int n, bool in_lds) {
    if (!in_lds) return;
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) g[e] = w[e];
    __syncthreads();
}

__device__ __forceinline__ double dscale(const SmallArgs& a, int j) { return j < a.r ? a.d[j] : 1.0; }

template <bool IN_LDS>
__global__ __launch_bounds__(SM_THREADS) void k_small_det1(SmallArgs a) {
    extern __shared__ __align__(16) double lds[];
    __shared__ int sflag;
    __shared__ int nonfinite;
    const int n = a.n, tid = threadIdx.x;
    constexpr bool in_lds = IN_LDS;
    double* W = in_lds ? lds : a.R1;
    // G <- D G' D, NaN/Inf check
    if (tid == 0) nonfinite = 0;
    __syncthreads();
    for (int e = tid; e < n * n; e += SM_THREADS) {
        const int i = e % n, j = e / n;
        const double v = a.G[e] * dscale(a, i) * dscale(a, j);
        if (!finite_d(v)) nonfinite = 1;
        a.G[e] = v;
        W[e] = v;
    }
    __syncthreads();
    if (nonfinite) {
        if (tid == 0) *a.status |= DEV_NONFINITE;
        return;
    }
    bool ok = wg_chol_upper(W, n, n);
    if (ok) {
        stage_out(W, a.R1, n, in_lds);
        double* X = (n <= SM_LDS_TWO_N) ? lds + (size_t)n * n : a.Ri;
        wg_trinv_upper(in_lds ? W : a.R1, n, n, X, n, in_lds ? lds_vecs(lds, n) : a.vec);
        // Ri and Xn = D R1^-1
        for (int e = tid; e < n * n; e += SM_THREADS) {
            const double v = X[e];
            a.Ri[e] = v;
            a.Xn[e] = v * dscale(a, e % n);
        }
        return;
    }
    if (!a.allow_fallback) {
        if (tid == 0) *a.status |= DEV_BREAKDOWN;
        return;
    }
    // Eigen route: the PSD Gram G = V diag(sigma^2) V^T by pivoted Cholesky
    // and one-sided Jacobi on its factor (wg_psd_eig: sigma_j is the j-th
    // singular value of the factor, so of the panel); U_new = C V_K diag(1 / sigma_K).
    if (tid == 0) *a.status |= DEV_FALLBACK;
    for (int e = tid; e < n * n; e += SM_THREADS) W[e] = a.G[e];
    __syncthreads();
    double* sig = in_lds ? lds_vecs(lds, n) : a.vec;
    double* nrm = sig + n;
    int* ord = in_lds ? (int*)(nrm + n + 1) : a.ivec;
    double* sv;
    int* col;
    int sw = wg_psd_eig(W, n, sig, nrm, ord, ord + n, ord + 2 * n, a.max_sweeps, &sflag, &sv, &col,
                        (double)n * 0x1p-53);
    if (tid == 0) {
        *a.sweeps = sw;
        if (sw > a.max_sweeps) *a.status |= DEV_NOCONV;
    }
    const int rk = a.K < n ? a.K : n;
    for (int e = tid; e < n * rk; e += SM_THREADS) {
        const int i = e % n, j = e / n;
        a.small_u[i + (size_t)j * n] = W[i + (size_t)col[j] * n];
    }
    for (int j = tid; j < rk; j += SM_THREADS) a.s_out[j] = sv[j];
    __syncthreads();
    wg_sign_rule(a.small_u, n, rk, n, nullptr);
    for (int e = tid; e < n * rk; e += SM_THREADS) {
        const int i = e % n, j = e / n;
        const double sj = a.s_out[j];
        a.T[i + (size_t)j * n] = sj > 0.0 ? dscale(a, i) * a.small_u[i + (size_t)j * n] / sj : 0.0;
    }
}

// After the second Gram G2 = Q1^T Q1: R2 = chol(G2), R = R2 R1, Jacobi SVD of
// R -> U~ (left vectors), S; sort, sign rule, keep rk = min(K, n);
// T = D R^-1 U~_rk.
template <bool IN_LDS>
__global__ __launch_bounds__(SM_THREADS) void k_small_det2(SmallArgs a) {
    extern __shared__ __align__(16) double lds[];
    __shared__ int sflag;
    if (*a.status & (DEV_FALLBACK | DEV_NONFINITE | DEV_BREAKDOWN)) return;
    const int n = a.n, tid = threadIdx.x;
    constexpr bool in_lds = IN_LDS;
    double* W = stage_in(lds, a.G2, n, in_lds);
    bool ok = wg_chol_upper(W, n, n);
    if (!ok) {
        // Q1 is orthonormal to working accuracy once the first factor exists;
        // a breakdown here means non-finite data.
        if (tid == 0) *a.status |= DEV_NONFINITE;
        return;
    }
    const bool two = n <= SM_LDS_TWO_N;
    double* R2 = two ? lds + (size_t)n * n : a.G2;     // R2 kept for the final solve
    for (int e = tid; e < n * n; e += SM_THREADS) {
        const double v = W[e];
        if (two) R2[e] = v;
        if (in_lds) a.G2[e] = v;
    }
    __syncthreads();
    // R = R2 R1 (upper) -> a.G (kept) and the working matrix; k ascending,
    // eight pairs of loads issued before their multiply-adds
    for (int e = tid; e < n * n; e += SM_THREADS) {
        const int i = e % n, j = e / n;
        double s = 0.0;
        int k = i;
        for (; k + 8 <= j + 1; k += 8) {
            double r2[8], r1[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                r2[u] = R2[i + (size_t)(k + u) * n];
                r1[u] = a.R1[k + u + (size_t)j * n];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) s += r2[u] * r1[u];
        }
        for (; k <= j; ++k) s += R2[i + (size_t)k * n] * a.R1[k + (size_t)j * n];
        a.G[e] = (i <= j) ? s : 0.0;
    }
    __syncthreads();
    if (a.skip_svd) return;
    W = in_lds ? lds : a.Z;
    for (int e = tid; e < n * n; e += SM_THREADS) W[e] = a.G[e];
    __syncthreads();
    double* sig = in_lds ? lds_vecs(lds, n) : a.vec;
    double* nrm = sig + n;
    int* ord = in_lds ? (int*)(nrm + n + 1) : a.ivec;
    int sw = wg_jacobi(W, n, n, n, sig, ord, nrm, a.max_sweeps, &sflag, nullptr, false, a.stop_cos2);
    if (tid == 0) {
        *a.sweeps = sw;
        if (sw > a.max_sweeps) *a.status |= DEV_NOCONV;
    }
    const int rk = a.K < n ? a.K : n;
    for (int e = tid; e < n * rk; e += SM_THREADS) {
        const int i = e % n, j = e / n;
        a.small_u[i + (size_t)j * n] = W[i + (size_t)ord[j] * n];
    }
    for (int j = tid; j < rk; j += SM_THREADS) a.s_out[j] = sig[ord[j]];
    __syncthreads();
    wg_sign_rule(a.small_u, n, rk, n, nullptr);
    // The lift reads Q1 = C D R1^-1 (the first Cholesky-QR factor, kept by the
    // second Gram pass): U = Q1 R2^-1 U~_rk, so T = R2^-1 U~ (row-step solve;
    // the working matrix is free again and holds the solution when in LDS).
    double* X = in_lds ? W : a.T;
    wg_trsm_upper(R2, n, n, a.small_u, n, X, n, rk);
    if (in_lds)
        for (int e = tid; e < n * rk; e += SM_THREADS) a.T[e] = X[e];
}

// ---------------------------------------------------------------------------
// Randomized-path small kernels (one work-group each; P, n x l, is the
// projection C^T Y or D C'^T (C' X) summed by the fused pass).
// ---------------------------------------------------------------------------

// Cholesky of the l x l Gram G (in LDS or global scratch W, copied from Gsrc)
// with the shifted retry of Fukaya et al. 2020 on breakdown: shift
// 11 (l^2 + l) 2^-53 ||G||_F on the diagonal, flag_bit set in the status.
// Returns false if the shifted factorisation fails too.
__device__ __forceinline__ bool chol_shifted(const double* Gsrc, double* W, int l, int32_t* status, int flag_bit, double* red,
                             double* S = nullptr) {
    const int tid = threadIdx.x;
    const bool fast = S != nullptr && l <= 64 && blockDim.x == 1024;   // S: 64 x 65 doubles of LDS
    if (fast) {
        if (wg_chol64b(Gsrc, l, 0.0, S, W)) return true;
    } else {
        for (int e = tid; e < l * l; e += blockDim.x) W[e] = Gsrc[e];
        __syncthreads();
        if (wg_chol_upper(W, l, l)) return true;
    }
    // ||G||_F by a fixed-order sum (per-thread partials, then thread 0)
    double f = 0.0;
    for (int e = tid; e < l * l; e += blockDim.x) f += Gsrc[e] * Gsrc[e];
    red[tid] = f;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int q = 0; q < (int)blockDim.x; ++q) t += red[q];
        red[0] = sqrt(t);
        *status |= flag_bit;
    }
    __syncthreads();
    const double shift = 11.0 * ((double)l * l + l) * 0x1p-53 * red[0];
    __syncthreads();
    if (fast) return wg_chol64b(Gsrc, l, shift, S, W);
    for (int e = tid; e < l * l; e += blockDim.x) {
        const int i = e % l, j = e / l;
        W[e] = Gsrc[e] + (i == j ? shift : 0.0);
    }
    __syncthreads();
    return wg_chol_upper(W, l, l);
}

// LDS of the randomized small kernels: two l x l matrices (the first with
// leading dimension 64 when l <= 64), 3 l + 8 vector entries and, for
// l <= 64, the chunk of the staged tall products.
__host__ __device__ inline size_t rand_lds_doubles(int l) {
    return l <= 64 ? 64 * (size_t)l + (size_t)l * l + 3 * (size_t)l + 8 + TALL_CHUNK
                   : 2 * (size_t)l * l + 3 * (size_t)l + 8;
}

// Power-iteration re-orthonormalisation X = D P R^-1 with R = chol(P^T P).
// When the randomized small kernels keep their matrices in global memory (l
// too large for two l x l matrices in LDS), their working matrix (the
// Cholesky factor; in the final core also R_b^T and its Jacobi) and the
// vectors still sit in LDS if one l x l matrix and 3 l + 8 doubles fit.
__host__ __device__ inline size_t rand_jac_lds_bytes(int l) {
    return ((size_t)l * l + 3 * (size_t)l + 8) * sizeof(double);
}
__host__ __device__ inline bool rand_jac_in_lds(int l) { return rand_jac_lds_bytes(l) <= 150 * 1024; }

template <bool IN_LDS>
__global__ __launch_bounds__(SM_THREADS) void k_small_orth(OrthArgs a) {
    extern __shared__ __align__(16) double lds[];
    __shared__ double red[SM_THREADS];
    if (*a.status & (DEV_NONFINITE | DEV_BREAKDOWN)) return;
    const int l = a.l, n = a.n;
    constexpr bool in_lds = IN_LDS;
    const bool staged = in_lds && l <= 64;
    const bool r_lds = in_lds || rand_jac_in_lds(l);
    double* R = r_lds ? lds : a.R;
    double* Ri = in_lds ? lds + (size_t)l * l : a.Ri;
    double* rinv = in_lds ? lds + 2 * (size_t)l * l : r_lds ? lds + (size_t)l * l : a.vec;
    double* Cn = lds + 2 * (size_t)l * l + 3 * (size_t)l + 8;
    // G = P^T P (global scratch, kept for the shifted retry)
    if (staged) wg_gram_tall(n, l, a.P, n, a.G, l, Cn);
    else wg_gemm_f64(l, l, n, a.P, n, 1, a.P, 1, n, a.G, 1, l, nullptr, 0);
    if (!chol_shifted(a.G, R, l, a.status, a.flag_bit, red, staged ? Cn : nullptr)) {
        if (threadIdx.x == 0) *a.status |= DEV_NONFINITE;
        return;
    }
    wg_trinv_upper(R, l, l, Ri, l, rinv);
    if (staged) wg_mul_tall(n, l, a.P, n, Ri, l, a.X, n, a.d, a.r, Cn);
    else wg_gemm_f64(n, l, l, a.P, 1, n, Ri, 1, l, a.X, 1, n, a.d, a.r);
}

// Everything after the final pass:
//   R_Y = chol(G_Y), R_Y^-1;  Cholesky-QR2 of P: R1 = chol(P^T P),
//   P1 = P R1^-1, R2 = chol(P1^T P1), R_P = R2 R1;  R_b = R_P R_Y^-1;
//   one-sided Jacobi on R_b^T -> U~ (left singular vectors of B = Q^T C),
//   S;  sort, sign rule, keep rk = min(K, l);  M2 = R_Y^-1 U~_rk.
template <bool IN_LDS>
__global__ __launch_bounds__(SM_THREADS) void k_small_rand_final(RandFinalArgs a) {
    extern __shared__ __align__(16) double lds[];
    __shared__ double red[SM_THREADS];
    __shared__ int sflag;
    if (*a.status & (DEV_NONFINITE | DEV_BREAKDOWN)) return;
    const int l = a.l, n = a.n, tid = threadIdx.x;
    constexpr bool in_lds = IN_LDS;
    const bool staged = in_lds && l <= 64;
    // staged: W spans 64 x l so that R_b^T can take leading dimension 64
    const size_t wsz = staged ? 64 * (size_t)l : (size_t)l * l;
    // global-memory form: the working matrix and the vectors still in LDS when they fit
    const bool w_lds = in_lds || rand_jac_in_lds(l);
    double* W = w_lds ? lds : a.W;                       // working l x l
    double* V = in_lds ? lds + wsz : a.V;                // second l x l
    double* vec = in_lds ? lds + wsz + (size_t)l * l : w_lds ? lds + (size_t)l * l : a.vec;   // 2 l + 1 doubles + l ints
    double* Cn = lds + wsz + (size_t)l * l + 3 * (size_t)l + 8;   // staging chunk (staged only)
    const int rk = a.K < l ? a.K : l;
    auto bail = [&]() {
        if (tid == 0) *a.status |= DEV_NONFINITE;
    };
    // R_Y and R_Y^-1 (V, copied out).  A breakdown of the Cholesky factorisation,
    // or a pivot with R_jj^2 <= l 2^-33 max_i (G_Y)_ii (Y numerically rank-
    // deficient: its Cholesky factor would carry errors of order one), takes
    // the eigen route below instead.
    bool chol_ok;
    if (staged) {
        chol_ok = wg_chol64b(a.GY, l, 0.0, Cn, W);
    } else {
        for (int e = tid; e < l * l; e += SM_THREADS) W[e] = a.GY[e];
        __syncthreads();
        chol_ok = wg_chol_upper(W, l, l);
    }
    if (chol_ok) {
        if (tid == 0) {
            double gmax = 0.0, pmin = INFINITY;
            for (int i = 0; i < l; ++i) {
                gmax = fmax(gmax, a.GY[i + (size_t)i * l]);
                const double rjj = W[i + (size_t)i * l];
                pmin = fmin(pmin, rjj * rjj);
            }
            sflag = pmin > (double)l * 0x1p-33 * gmax;
        }
        __syncthreads();
        chol_ok = sflag != 0;
        __syncthreads();
    }
    if (!chol_ok) {
        // Eigen route: G_Y = V diag(lambda) V^T by one-sided Jacobi; the columns
        // v_j / sqrt(lambda_j) of the eigenpairs above the floor l 2^-33 lambda_max
        // (descending) replace R_Y^-1, so Q = Y R_Y^-1 is an orthonormal basis of
        // the numerical range of Y and its null directions drop out.  Then
        // B = Q^T C = (P W_r)^T: Cholesky QR of P W_r, SVD of its R factor.
        if (tid == 0) *a.status |= DEV_FALLBACK;
        for (int e = tid; e < l * l; e += SM_THREADS) W[e] = a.GY[e];
        __syncthreads();
        double* sig = vec;
        double* nrm = sig + l;
        int* ord = (int*)(nrm + l + 1);
        const int swe = wg_jacobi(W, l, l, l, sig, ord, nrm, a.max_sweeps, &sflag);
        if (tid == 0 && swe > a.max_sweeps) *a.status |= DEV_NOCONV;
        const double floor_l = (double)l * 0x1p-33 * sig[ord[0]];
        int rr = 0;
        for (int k = 0; k < l; ++k) rr += sig[ord[k]] > floor_l ? 1 : 0;
        for (int e = tid; e < l * l; e += SM_THREADS) {
            const int i = e % l, k = e / l;
            const double lam = sig[ord[k]];
            a.RYi[e] = k < rr ? W[i + (size_t)ord[k] * l] / sqrt(lam) : 0.0;
            a.RY[e] = 0.0;
        }
        __syncthreads();
        // P1 = P W_r (n x rr), G1 = P1^T P1, R1 = chol(G1)
        wg_gemm_f64(n, rr, l, a.P, 1, n, a.RYi, 1, l, a.P1, 1, n, nullptr, 0);
        wg_gemm_f64(rr, rr, n, a.P1, n, 1, a.P1, 1, n, a.G1, 1, rr, nullptr, 0);
        if (!chol_shifted(a.G1, a.R1, rr, a.status, DEV_FALLBACK, red, nullptr)) return bail();
        // Z = R1^T (rr x rr) -> left singular vectors of B, singular values
        for (int e = tid; e < rr * rr; e += SM_THREADS) {
            const int i = e % rr, j = e / rr;
            W[e] = a.R1[j + (size_t)i * rr];
        }
        __syncthreads();
        const int sw = wg_jacobi(W, rr, rr, rr, sig, ord, nrm, a.max_sweeps, &sflag);
        if (tid == 0) {
            *a.sweeps = sw;
            if (sw > a.max_sweeps) *a.status |= DEV_NOCONV;
        }
        const int rq = rk < rr ? rk : rr;
        // U~ (rr x rq) -> V, sign rule, M2 = W_r U~ (l x rq), zero columns past rq
        for (int e = tid; e < rr * rq; e += SM_THREADS) {
            const int i = e % rr, j = e / rr;
            V[i + (size_t)j * rr] = W[i + (size_t)ord[j] * rr];
        }
        for (int j = tid; j < rk; j += SM_THREADS) a.s_out[j] = j < rq ? sig[ord[j]] : 0.0;
        __syncthreads();
        wg_sign_rule(V, rr, rq, rr, nullptr);
        for (int e = tid; e < l * rk; e += SM_THREADS) {
            const int i = e % l, j = e / l;
            a.small_u[e] = (i < rr && j < rq) ? V[i + (size_t)j * rr] : 0.0;
        }
        for (int e = tid; e < l * rk; e += SM_THREADS) a.M2[e] = 0.0;
        __syncthreads();
        if (rq > 0) wg_gemm_f64(l, rq, rr, a.RYi, 1, l, V, 1, rr, a.M2, 1, l, nullptr, 0);
        return;
    }
    for (int e = tid; e < l * l; e += SM_THREADS) a.RY[e] = W[e];
    wg_trinv_upper(W, l, l, V, l, vec);
    for (int e = tid; e < l * l; e += SM_THREADS) a.RYi[e] = V[e];
    // R1 = chol(P^T P)
    if (staged) wg_gram_tall(n, l, a.P, n, a.G1, l, Cn);
    else wg_gemm_f64(l, l, n, a.P, n, 1, a.P, 1, n, a.G1, 1, l, nullptr, 0);
    if (!chol_shifted(a.G1, W, l, a.status, DEV_FALLBACK, red, staged ? Cn : nullptr)) return bail();
    const double* RYi = a.RYi;
    if (a.qr_passes == 2) {
        // Cholesky-QR2: R1^-1 (V), P1 = P R1^-1, R2 = chol(P1^T P1) in W, R_P = R2 R1 -> V
        for (int e = tid; e < l * l; e += SM_THREADS) a.R1[e] = W[e];
        wg_trinv_upper(W, l, l, V, l, vec);
        if (staged) wg_mul_tall(n, l, a.P, n, V, l, a.P1, n, nullptr, 0, Cn);
        else wg_gemm_f64(n, l, l, a.P, 1, n, V, 1, l, a.P1, 1, n, nullptr, 0);
        if (staged) wg_gram_tall(n, l, a.P1, n, W, l, Cn);
        else wg_gemm_f64(l, l, n, a.P1, n, 1, a.P1, 1, n, W, 1, l, nullptr, 0);
        if (!(staged ? wg_chol64b(W, l, 0.0, Cn, W) : wg_chol_upper(W, l, l))) return bail();
        // small operands are read from LDS: R1 goes to the chunk buffer
        const double* R1 = a.R1;
        if (staged) {
            for (int e = tid; e < l * l; e += SM_THREADS) Cn[e] = a.R1[e];
            __syncthreads();
            R1 = Cn;
        }
        wg_gemm_f64(l, l, l, W, 1, l, R1, 1, l, V, 1, l, nullptr, 0);
    } else {
        // one Cholesky-QR pass: R_P = R1 -> V
        for (int e = tid; e < l * l; e += SM_THREADS) V[e] = W[e];
        __syncthreads();
    }
    // W = R_b^T = (R_P R_Y^-1)^T; R_Y^-1 is read from the chunk buffer
    if (staged) {
        for (int e = tid; e < l * l; e += SM_THREADS) Cn[e] = a.RYi[e];
        __syncthreads();
        RYi = Cn;
    }
    const int ldw = staged ? 64 : l;
    if (staged) {   // rows l..63 of the padded W are zero
        for (int e = tid; e < 64 * l; e += SM_THREADS) W[e] = 0.0;
        __syncthreads();
    }
    wg_gemm_f64(l, l, l, V, 1, l, RYi, 1, l, W, ldw, 1, nullptr, 0);
    double* Wj = W;
    double* vj = vec;
    double* sig = vj;
    double* nrm = sig + l;
    int* ord = (int*)(nrm + l + 1);
    const int sw = staged ? wg_jacobi_pad64(Wj, l, l, sig, ord, nrm, a.max_sweeps, &sflag, red, a.stop_cos2)
                          : wg_jacobi(Wj, l, l, l, sig, ord, nrm, a.max_sweeps, &sflag, nullptr, true);
    if (tid == 0) {
        *a.sweeps = sw;
        if (sw > a.max_sweeps) *a.status |= DEV_NOCONV;
    }
    // U~_rk (sorted, sign rule) -> V (l x rk) and small_u; M2 = R_Y^-1 U~_rk
    double* Us = in_lds ? V : a.small_u;
    for (int e = tid; e < l * rk; e += SM_THREADS) {
        const int i = e % l, j = e / l;
        Us[i + (size_t)j * l] = Wj[i + (size_t)ord[j] * ldw];
    }
    for (int j = tid; j < rk; j += SM_THREADS) a.s_out[j] = sig[ord[j]];
    __syncthreads();
    wg_sign_rule(Us, l, rk, l, nullptr);
    if (in_lds)
        for (int e = tid; e < l * rk; e += SM_THREADS) a.small_u[e] = Us[e];
    wg_gemm_f64(l, rk, l, RYi, 1, l, Us, 1, l, a.M2, 1, l, nullptr, 0);
}

// Asynchronous updates: fold the status word of the update into the sticky
// word read at the next synchronising call (st[2] errors, st[3] sweeps of the
// last small SVD, st[4] count of Cholesky fallbacks).
__global__ void k_status_fold(int32_t* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st[2] |= st[0] & ~(int32_t)DEV_FALLBACK;
        st[3] = st[1];
        if (st[0] & DEV_FALLBACK) st[4] += 1;
    }
}

// Row scaling of a small n x m matrix: rows i < r multiplied by d[i] (x mult times).
__global__ void k_scale_rows(double* X, int n, int m, int ldx, const double* d, int r, int times) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * m) return;
    int i = e % n, j = e / n;
    if (i < r) {
        double f = d[i];
        double v = X[i + (size_t)j * ldx];
        for (int t = 0; t < times; ++t) v *= f;
        X[i + (size_t)j * ldx] = v;
    }
}

// Start of a randomized update, one launch: the status words are cleared,
// d[j] = ff s[j] (j < r) and X = D Omega (rows i < r of the n x l test matrix
// multiplied by d[i]; Omega and X column-major with leading dimension n).
__global__ void k_rand_begin(int32_t* st, double* d, const double* s, int r, double ff, double* X,
                             const double* Om, int n, int l) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0) {
        st[0] = 0;
        st[1] = 0;
    }
    if (e < r) d[e] = ff * s[e];
    if (e < n * l) {
        const int i = e % n;
        const double v = Om[e];
        X[e] = i < r ? (ff * s[i]) * v : v;
    }
}

// Start of a deterministic update: the status words are cleared (st may be
// null) and d[j] = ff * s[j].
__global__ void k_make_scale(int32_t* st, double* d, const double* s, int r, double ff) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0 && st != nullptr) {
        st[0] = 0;
        st[1] = 0;
    }
    if (j < r) d[j] = ff * s[j];
}

// ---------------------------------------------------------------------------
// The low-rank SVD of a small matrix where the paper randomizes the parallel
// variant (the SVD of W in Algorithm 2, of the combined R factor in the
// partitioned update): Eqs. (7)-(11) without power iterations, one work-group,
// FP64, everything in global scratch.
//   Y = A Om (m x l);  Q = Y R^-1 by Cholesky QR twice (Q spans range(Y));
//   B^T = A^T Q (n x l);  one-sided Jacobi on the columns of B^T gives
//   B^T Z = W diag(s) with W the right singular vectors of B; the left ones
//   are U~ = B W diag(1 / s) = (B^T)^T W diag(1 / s);  sort, sign rule on U~;
//   U = Q U~[:, :k], k = min(K, l).
// ---------------------------------------------------------------------------
size_t low_rank_work_doubles(int m, int n, int l) {
    const size_t ll = (size_t)l * l;
    return (size_t)m * l + 3 * (size_t)n * l + 4 * ll + 4 * (size_t)(m > n ? m : n) + 4 * (size_t)l + 64;
}

__global__ __launch_bounds__(SM_THREADS) void k_low_rank_small(LowRankArgs a) {
    __shared__ double red[SM_THREADS];
    __shared__ int sflag;
    if (*a.status & (DEV_FALLBACK | DEV_NONFINITE | DEV_BREAKDOWN)) return;
    const int m = a.m, n = a.n, l = a.l, tid = threadIdx.x;
    const int k = a.K < l ? a.K : l;
    const size_t ll = (size_t)l * l;
    double* Y = a.work;                          // m x l: Y, then Q
    double* Bt = Y + (size_t)m * l;              // n x l
    double* Z = Bt + (size_t)n * l;              // n x l (Jacobi work)
    double* Zs = Z + (size_t)n * l;              // n x l (sorted right vectors)
    double* G = Zs + (size_t)n * l;              // l x l
    double* R = G + ll;                          // l x l
    double* Ri = R + ll;                         // l x l
    double* Ub = Ri + ll;                        // l x l
    double* vec = Ub + ll;                       // sig, nrm, ord, rinv
    double* sig = vec;
    double* nrm = sig + (m > n ? m : n);
    int* ord = (int*)(nrm + (m > n ? m : n) + 1);
    double* rinv = (double*)(ord + (m > n ? m : n) + 2);
    // Y = A Om
    wg_gemm_f64(m, l, n, a.A, (int)a.a_i, (int)a.a_j, a.Om, 1, n, Y, 1, m, nullptr, 0);
    // Q: two Cholesky-QR passes on Y (Bt holds the intermediate factor)
    for (int pass = 0; pass < 2; ++pass) {
        double* src = pass == 0 ? Y : Bt;
        double* dst = pass == 0 ? Bt : Y;
        wg_gemm_f64(l, l, m, src, m, 1, src, 1, m, G, 1, l, nullptr, 0);
        // (a shifted retry raises no status bit here: the callers' later kernels
        // test DEV_FALLBACK for the eigen route of the Cholesky QR of the panel)
        if (!chol_shifted(G, R, l, a.status, 0, red, nullptr)) {
            if (tid == 0) *a.status |= DEV_NONFINITE;
            return;
        }
        wg_trinv_upper(R, l, l, Ri, l, rinv);
        wg_gemm_f64(m, l, l, src, 1, m, Ri, 1, l, dst, 1, m, nullptr, 0);
    }
    // B^T = A^T Q, kept, and a working copy for the Jacobi SVD
    wg_gemm_f64(n, l, m, a.A, (int)a.a_j, (int)a.a_i, Y, 1, m, Bt, 1, n, nullptr, 0);
    for (int e = tid; e < n * l; e += SM_THREADS) Z[e] = Bt[e];
    __syncthreads();
    const int sw = wg_jacobi(Z, n, l, n, sig, ord, nrm, a.max_sweeps, &sflag);
    if (tid == 0) {
        atomicMax(a.sweeps, sw);
        if (sw > a.max_sweeps) *a.status |= DEV_NOCONV;
    }
    for (int e = tid; e < n * k; e += SM_THREADS) {
        const int i = e % n, j = e / n;
        Zs[i + (size_t)j * n] = Z[i + (size_t)ord[j] * n];
    }
    for (int j = tid; j < k; j += SM_THREADS) a.s[j] = sig[ord[j]];
    __syncthreads();
    // U~ = (B^T)^T W_k diag(1 / s)
    wg_gemm_f64(l, k, n, Bt, n, 1, Zs, 1, n, Ub, 1, l, nullptr, 0);
    for (int e = tid; e < l * k; e += SM_THREADS) {
        const double sj = a.s[e / l];
        Ub[e] = sj > 0.0 ? Ub[e] / sj : 0.0;
    }
    __syncthreads();
    wg_sign_rule(Ub, l, k, l, nullptr);
    wg_gemm_f64(m, k, l, Y, 1, m, Ub, 1, l, a.U, 1, (int)a.ldu, nullptr, 0);
    if (a.post == 1) {
        wg_trsm_upper(a.post_R, m, m, a.U, (int)a.ldu, a.T, m, k);
    } else if (a.post == 2) {
        if (tid == 0 && !(a.s[k - 1] > (double)n * 0x1p-53 * a.s[0])) *a.status |= DEV_SMALL_LAMBDA;
        for (int e = tid; e < m * k; e += SM_THREADS) {
            const int i = e % m, j = e / m;
            const double sj = a.s[j];
            a.T[e] = sj > 0.0 ? a.U[i + (size_t)j * a.ldu] / sj : 0.0;
        }
    }
}

hipError_t launch_low_rank_small(const LowRankArgs& a, hipStream_t st) {
    if (a.m < 1 || a.n < 1 || a.l < 1 || a.l > a.m || a.l > a.n || a.K < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_low_rank_small, dim3(1), dim3(SM_THREADS), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// APMOS small kernels.
// ---------------------------------------------------------------------------

// One work-group per partition: eigen-decomposition of G_i (wg_psd_eig);
// W_i = V_i[:, :r] diag(sqrt(lambda_i[:r])) stored transposed.
template <bool IN_LDS>
__global__ __launch_bounds__(SM_THREADS) void k_apmos_local(ApmosLocalArgs a) {
    extern __shared__ __align__(16) double lds[];
    __shared__ int sflag;
    const int i = blockIdx.x, N = a.N, tid = threadIdx.x;
    constexpr bool in_lds = IN_LDS;
    double* G = stage_in(lds, a.G + (size_t)i * N * N, N, in_lds);
    double* sig = in_lds ? lds_vecs(lds, N) : a.vec + (size_t)i * (2 * N + 2);
    double* nrm = sig + N;
    int* ord = in_lds ? (int*)(nrm + N + 1) : a.ivec + (size_t)i * 3 * N;
    double* sv;
    int* col;
    int sw = wg_psd_eig(G, N, sig, nrm, ord, ord + N, ord + 2 * N, a.max_sweeps, &sflag, &sv, &col,
                        (double)N * (a.data_f32 ? 0x1p-48 : 0x1p-53));
    if (tid == 0 && sw > a.max_sweeps) atomicOr(a.status, (int)DEV_NOCONV);
    if (tid == 0) atomicMax(a.sweeps, sw);
    const int ldw = a.P * a.r;
    for (int e = tid; e < N * a.r; e += SM_THREADS) {
        int k = e % N, j = e / N;
        a.Wt[(size_t)(i * a.r + j) + (size_t)k * ldw] = G[k + (size_t)col[j] * N] * sv[j];
    }
}


// W W^T = X Lambda^2 X^T (wg_psd_eig); keep K; sign rule on X~;
// T = X~ diag(1 / Lambda~) with the guard Lambda~_K > N 2^-53 Lambda~_1.
template <bool IN_LDS>
__global__ __launch_bounds__(SM_THREADS) void k_apmos_global(ApmosGlobalArgs a) {
    extern __shared__ __align__(16) double lds[];
    __shared__ int sflag;
    const int N = a.N, tid = threadIdx.x;
    constexpr bool in_lds = IN_LDS;
    double* WW = stage_in(lds, a.WW, N, in_lds);
    double* sig = in_lds ? lds_vecs(lds, N) : a.vec;
    double* nrm = sig + N;
    int* ordv = in_lds ? (int*)(nrm + N + 1) : a.ivec;
    double* sv;
    int* col;
    int sw = wg_psd_eig(WW, N, sig, nrm, ordv, ordv + N, ordv + 2 * N, a.max_sweeps, &sflag, &sv, &col,
                        (double)N * 0x1p-53);
    if (tid == 0) {
        atomicMax(a.sweeps, sw);
        if (sw > a.max_sweeps) *a.status |= DEV_NOCONV;
    }
    for (int e = tid; e < N * a.K; e += SM_THREADS) {
        int k = e % N, j = e / N;
        a.X[k + (size_t)j * N] = WW[k + (size_t)col[j] * N];
    }
    for (int j = tid; j < a.K; j += SM_THREADS) a.Lam[j] = sv[j];
    __syncthreads();
    wg_sign_rule(a.X, N, a.K, N, nullptr);
    if (tid == 0 && !(a.Lam[a.K - 1] > (double)N * 0x1p-53 * a.Lam[0])) *a.status |= DEV_SMALL_LAMBDA;
    for (int e = tid; e < N * a.K; e += SM_THREADS) {
        int j = e / N;
        double lj = a.Lam[j];
        a.T[e] = lj > 0.0 ? a.X[e] / lj : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
hipError_t launch_small_det1(const SmallArgs& a, hipStream_t st) {
    size_t lds = small_lds_bytes(a.n);
    const bool in_lds = (a.n) <= SM_LDS_MAX_N;
    const void* fn = in_lds ? (const void*)k_small_det1<true> : (const void*)k_small_det1<false>;
    hipError_t e = ensure_lds_attr(fn, lds);
    if (e != hipSuccess) return e;
    if (in_lds) hipLaunchKernelGGL(k_small_det1<true>, dim3(1), dim3(SM_THREADS), lds, st, a);
    else hipLaunchKernelGGL(k_small_det1<false>, dim3(1), dim3(SM_THREADS), lds, st, a);
    return hipGetLastError();
}
hipError_t launch_small_det2(const SmallArgs& a, hipStream_t st) {
    size_t lds = small_lds_bytes(a.n);
    const bool in_lds = (a.n) <= SM_LDS_MAX_N;
    const void* fn = in_lds ? (const void*)k_small_det2<true> : (const void*)k_small_det2<false>;
    hipError_t e = ensure_lds_attr(fn, lds);
    if (e != hipSuccess) return e;
    if (in_lds) hipLaunchKernelGGL(k_small_det2<true>, dim3(1), dim3(SM_THREADS), lds, st, a);
    else hipLaunchKernelGGL(k_small_det2<false>, dim3(1), dim3(SM_THREADS), lds, st, a);
    return hipGetLastError();
}
// LDS of the randomized small kernels: two l x l matrices and 3 l vectors.
static size_t rand_lds_bytes(int l) { return rand_lds_doubles(l) * sizeof(double); }
static bool rand_in_lds(int l) { return rand_lds_bytes(l) <= 150 * 1024; }

hipError_t launch_small_orth(const OrthArgs& a, hipStream_t st) {
    const bool in_lds = rand_in_lds(a.l);
    const size_t lds = in_lds ? rand_lds_bytes(a.l) : rand_jac_in_lds(a.l) ? rand_jac_lds_bytes(a.l) : 64;
    const void* fn = in_lds ? (const void*)k_small_orth<true> : (const void*)k_small_orth<false>;
    hipError_t e = ensure_lds_attr(fn, lds);
    if (e != hipSuccess) return e;
    if (in_lds) hipLaunchKernelGGL(k_small_orth<true>, dim3(1), dim3(SM_THREADS), lds, st, a);
    else hipLaunchKernelGGL(k_small_orth<false>, dim3(1), dim3(SM_THREADS), lds, st, a);
    return hipGetLastError();
}
hipError_t launch_small_rand_final(const RandFinalArgs& a, hipStream_t st) {
    const bool in_lds = rand_in_lds(a.l);
    const size_t lds = in_lds ? rand_lds_bytes(a.l) : rand_jac_in_lds(a.l) ? rand_jac_lds_bytes(a.l) : 64;
    const void* fn = in_lds ? (const void*)k_small_rand_final<true> : (const void*)k_small_rand_final<false>;
    hipError_t e = ensure_lds_attr(fn, lds);
    if (e != hipSuccess) return e;
    if (in_lds) hipLaunchKernelGGL(k_small_rand_final<true>, dim3(1), dim3(SM_THREADS), lds, st, a);
    else hipLaunchKernelGGL(k_small_rand_final<false>, dim3(1), dim3(SM_THREADS), lds, st, a);
    return hipGetLastError();
}
hipError_t launch_status_fold(int32_t* st, hipStream_t stream) {
    hipLaunchKernelGGL(k_status_fold, dim3(1), dim3(64), 0, stream, st);
    return hipGetLastError();
}
hipError_t launch_scale_rows(double* X, int n, int m, int ldx, const double* d, int r, int times, hipStream_t st) {
    if (r <= 0 || n * m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_rows, dim3((n * m + 255) / 256), dim3(256), 0, st, X, n, m, ldx, d, r, times);
    return hipGetLastError();
}
hipError_t launch_rand_begin(int32_t* status, double* d, const double* s, int r, double ff, double* X,
                             const double* Om, int n, int l, hipStream_t st) {
    const int total = n * l > r ? n * l : (r > 0 ? r : 1);
    hipLaunchKernelGGL(k_rand_begin, dim3((total + 255) / 256), dim3(256), 0, st, status, d, s, r, ff, X, Om, n, l);
    return hipGetLastError();
}
hipError_t launch_make_scale(int32_t* status, double* d, const double* s, int r, double ff, hipStream_t st) {
    if (r <= 0 && status == nullptr) return hipSuccess;
    hipLaunchKernelGGL(k_make_scale, dim3(((r > 0 ? r : 1) + 255) / 256), dim3(256), 0, st, status, d, s, r, ff);
    return hipGetLastError();
}
hipError_t launch_apmos_local(const ApmosLocalArgs& a, hipStream_t st) {
    size_t lds = small_lds_bytes(a.N);
    const bool in_lds = (a.N) <= SM_LDS_MAX_N;
    const void* fn = in_lds ? (const void*)k_apmos_local<true> : (const void*)k_apmos_local<false>;
    hipError_t e = ensure_lds_attr(fn, lds);
    if (e != hipSuccess) return e;
    if (in_lds) hipLaunchKernelGGL(k_apmos_local<true>, dim3(a.P), dim3(SM_THREADS), lds, st, a);
    else hipLaunchKernelGGL(k_apmos_local<false>, dim3(a.P), dim3(SM_THREADS), lds, st, a);
    return hipGetLastError();
}
hipError_t launch_apmos_global(const ApmosGlobalArgs& a, hipStream_t st) {
    size_t lds = small_lds_bytes(a.N);
    const bool in_lds = (a.N) <= SM_LDS_MAX_N;
    const void* fn = in_lds ? (const void*)k_apmos_global<true> : (const void*)k_apmos_global<false>;
    hipError_t e = ensure_lds_attr(fn, lds);
    if (e != hipSuccess) return e;
    if (in_lds) hipLaunchKernelGGL(k_apmos_global<true>, dim3(1), dim3(SM_THREADS), lds, st, a);
    else hipLaunchKernelGGL(k_apmos_global<false>, dim3(1), dim3(SM_THREADS), lds, st, a);
    return hipGetLastError();
}

}  // namespace psvd
