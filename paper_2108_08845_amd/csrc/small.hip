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
// Returns false (uniformly) on a non-positive or non-finite pivot.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool wg_chol_upper(double* A, int n, int lda, int* sflag) {
    // Right-looking, one barrier per column: every thread recomputes
    // r_kk = sqrt(a_kk) and scales the row-k entries it reads, the thread that
    // owns (k, j) stores r_kj, and the trailing (i, j) entries are updated in
    // the same step (a_ij -= a_ki a_kj / a_kk).
    const int tid = threadIdx.x;
    if (tid == 0) *sflag = 0;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double d = A[k + (size_t)k * lda];
        if (!(d > 0.0) || !finite_d(d)) {
            if (tid == 0) *sflag = 1;
            __syncthreads();
            return false;
        }
        const double rkk = sqrt(d);
        const double inv = 1.0 / rkk;
        const int m = n - k;            // columns k .. n-1 of row k, and the trailing block
        // trailing block (k < i <= j) and row k (i == k) in one sweep over (i, j), i, j >= k
        for (int e = tid; e < m * m; e += blockDim.x) {
            const int i = k + e % m, j = k + e / m;
            if (i > j) continue;
            if (i == k) continue;   // row k is written after the barrier (still read here)
            A[i + (size_t)j * lda] -= A[k + (size_t)i * lda] * A[k + (size_t)j * lda] * (inv * inv);
        }
        __syncthreads();
        for (int j = k + tid; j < n; j += blockDim.x) A[k + (size_t)j * lda] = (j == k) ? rkk : A[k + (size_t)j * lda] * inv;
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e % n, j = e / n;
        if (i > j) A[i + (size_t)j * lda] = 0.0;
    }
    __syncthreads();
    return true;
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

// Ri = R^-1 for upper triangular R (n x n).
__device__ __forceinline__ void wg_trinv_upper(const double* R, int n, int ldr, double* Ri, int ldi) {
    wg_trsm_upper(R, ldr, n, nullptr, 0, Ri, ldi, n);
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
// One-sided Jacobi on the columns of Z (m x n, ldz), in place.  On return
// the columns are mutually orthogonal to the tolerance m * 2^-53; sig[j] =
// ||z_j|| and z_j /= sig[j] (0 columns stay 0).  order[0..n) lists the
// columns by descending sig (stable).  Parallel round-robin ordering: each
// round rotates n/2 disjoint pairs, one pair per wave at a time.
// Returns the number of sweeps (> max_sweeps: not converged).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double q16_sum(double v) {
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 16);
    return v;
}

__device__ __forceinline__ int wg_jacobi(double* Z, int m, int n, int ldz, double* sig, int* order, double* nrm,
                                         int max_sweeps, int* sflag) {
    // One pair per quarter-wave (16 lanes): a round of n/2 disjoint pairs runs
    // in one pass when blockDim.x / 16 >= n / 2.
    const int tid = threadIdx.x;
    const int ql = tid & 15, qw = tid >> 4, nq = blockDim.x >> 4;
    const double tol = (double)m * 0x1p-53;
    const int ne = n + (n & 1);
    int sweep = 0;
    for (;;) {
        for (int j = qw; j < n; j += nq) {
            const double* z = Z + (size_t)j * ldz;
            double s = 0.0;
            for (int i = ql; i < m; i += 16) s += z[i] * z[i];
            s = q16_sum(s);
            if (ql == 0) nrm[j] = s;
        }
        if (tid == 0) *sflag = 0;
        __syncthreads();
        double nmax = 0.0;
        for (int j = 0; j < n; ++j) nmax = fmax(nmax, nrm[j]);
        const double negl = nmax * tol * tol;
        if (sweep >= max_sweeps) {
            ++sweep;
            break;
        }
        for (int t = 0; t < ne - 1; ++t) {
            for (int pi = qw; pi < ne / 2; pi += nq) {
                const int pa = pi, pb = ne - 1 - pi;
                const int ca = pa == 0 ? 0 : 1 + (pa - 1 + t) % (ne - 1);
                const int cb = pb == 0 ? 0 : 1 + (pb - 1 + t) % (ne - 1);
                const int p = ca < cb ? ca : cb, q = ca < cb ? cb : ca;
                if (q >= n) continue;
                double* zp = Z + (size_t)p * ldz;
                double* zq = Z + (size_t)q * ldz;
                double g = 0.0;
                for (int i = ql; i < m; i += 16) g += zp[i] * zq[i];
                g = q16_sum(g);
                const double al = nrm[p], be = nrm[q];
                if (!(al > negl) || !(be > negl)) continue;
                if (fabs(g) <= tol * sqrt(al) * sqrt(be)) continue;
                const double zeta = (be - al) / (2.0 * g);
                const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
                for (int i = ql; i < m; i += 16) {
                    const double a = zp[i], b = zq[i];
                    zp[i] = c * a - s * b;
                    zq[i] = s * a + c * b;
                }
                if (ql == 0) {
                    nrm[p] = al - tt * g;
                    nrm[q] = be + tt * g;
                    *sflag = 1;
                }
            }
            __syncthreads();
        }
        ++sweep;
        const int rotated = *sflag;
        __syncthreads();
        if (!rotated) break;
    }
    // singular values, normalisation
    for (int j = qw; j < n; j += nq) {
        double* z = Z + (size_t)j * ldz;
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
    extern __shared__ double lds[];
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
    bool ok = wg_chol_upper(W, n, n, &sflag);
    if (ok) {
        stage_out(W, a.R1, n, in_lds);
        double* X = (n <= SM_LDS_TWO_N) ? lds + (size_t)n * n : a.Ri;
        wg_trinv_upper(in_lds ? W : a.R1, n, n, X, n);
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
    // Eigen route: one-sided Jacobi on the PSD Gram G = V diag(lambda) V^T
    // (G V has orthogonal columns lambda_j v_j); sigma_j = sqrt(lambda_j),
    // U_new = C V_K diag(1 / sigma_K).
    if (tid == 0) *a.status |= DEV_FALLBACK;
    for (int e = tid; e < n * n; e += SM_THREADS) W[e] = a.G[e];
    __syncthreads();
    double* sig = in_lds ? lds_vecs(lds, n) : a.vec;
    double* nrm = sig + n;
    int* ord = in_lds ? (int*)(nrm + n) : a.ivec;
    int sw = wg_jacobi(W, n, n, n, sig, ord, nrm, a.max_sweeps, &sflag);
    if (tid == 0) {
        *a.sweeps = sw;
        if (sw > a.max_sweeps) *a.status |= DEV_NOCONV;
    }
    const int rk = a.K < n ? a.K : n;
    for (int e = tid; e < n * rk; e += SM_THREADS) {
        const int i = e % n, j = e / n;
        a.small_u[i + (size_t)j * n] = W[i + (size_t)ord[j] * n];
    }
    for (int j = tid; j < rk; j += SM_THREADS) {
        const double lam = sig[ord[j]];
        a.s_out[j] = sqrt(lam > 0.0 ? lam : 0.0);
    }
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
    extern __shared__ double lds[];
    __shared__ int sflag;
    if (*a.status & (DEV_FALLBACK | DEV_NONFINITE | DEV_BREAKDOWN)) return;
    const int n = a.n, tid = threadIdx.x;
    constexpr bool in_lds = IN_LDS;
    double* W = stage_in(lds, a.G2, n, in_lds);
    bool ok = wg_chol_upper(W, n, n, &sflag);
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
    // R = R2 R1 (upper) -> a.G (kept) and the working matrix
    for (int e = tid; e < n * n; e += SM_THREADS) {
        const int i = e % n, j = e / n;
        double s = 0.0;
        for (int k = i; k <= j; ++k) s += R2[i + (size_t)k * n] * a.R1[k + (size_t)j * n];
        a.G[e] = (i <= j) ? s : 0.0;
    }
    __syncthreads();
    W = in_lds ? lds : a.Z;
    for (int e = tid; e < n * n; e += SM_THREADS) W[e] = a.G[e];
    __syncthreads();
    double* sig = in_lds ? lds_vecs(lds, n) : a.vec;
    double* nrm = sig + n;
    int* ord = in_lds ? (int*)(nrm + n) : a.ivec;
    int sw = wg_jacobi(W, n, n, n, sig, ord, nrm, a.max_sweeps, &sflag);
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
// Randomized-path small kernels.
// ---------------------------------------------------------------------------

// R = chol(H) (R overwrites H), Ri = R^-1.  On breakdown a diagonal shift
// s = 11 (l^2 + l) 2^-53 ||H||_F (shifted Cholesky-QR of Fukaya et al. 2020)
// is added and the factorisation repeated.
template <bool IN_LDS>
__global__ __launch_bounds__(256) void k_small_chol(CholArgs a) {
    extern __shared__ double lds[];
    __shared__ int sflag;
    __shared__ double fro;
    const int l = a.l, tid = threadIdx.x;
    if (*a.status & (DEV_NONFINITE | DEV_BREAKDOWN)) return;
    constexpr bool in_lds = IN_LDS;
    double* W = in_lds ? lds : a.Ri;   // global fallback works in Ri and keeps H for the retry
    for (int e = tid; e < l * l; e += blockDim.x) W[e] = a.H[e];
    __syncthreads();
    bool ok = wg_chol_upper(W, l, l, &sflag);
    if (!ok) {
        if (tid == 0) {
            double f = 0.0;
            for (int e = 0; e < l * l; ++e) f += a.H[e] * a.H[e];
            fro = sqrt(f);
            *a.status |= a.flag_bit;
        }
        __syncthreads();
        const double shift = 11.0 * ((double)l * l + l) * 0x1p-53 * fro;
        for (int e = tid; e < l * l; e += blockDim.x) {
            const int i = e % l, j = e / l;
            W[e] = a.H[e] + (i == j ? shift : 0.0);
        }
        __syncthreads();
        ok = wg_chol_upper(W, l, l, &sflag);
        if (!ok) {
            if (tid == 0) *a.status |= DEV_NONFINITE;
            return;
        }
    }
    for (int e = tid; e < l * l; e += blockDim.x) a.H[e] = W[e];
    __syncthreads();
    if (l <= SM_LDS_TWO_N) {
        double* X = lds + (size_t)l * l;
        wg_trinv_upper(W, l, l, X, l);
        for (int e = tid; e < l * l; e += blockDim.x) a.Ri[e] = X[e];
    } else {
        wg_trinv_upper(in_lds ? W : a.H, l, l, a.Ri, l);
    }
}

// R_P = chol(H2) R1 (QR factor of P); R_b = R_P R_Y^-1; the left singular
// vectors of B = R_Y^-T P^T are those of R_b^T: one-sided Jacobi on R_b^T.
template <bool IN_LDS>
__global__ __launch_bounds__(SM_THREADS) void k_small_rand_final(RandFinalArgs a) {
    extern __shared__ double lds[];
    __shared__ int sflag;
    if (*a.status & (DEV_NONFINITE | DEV_BREAKDOWN)) return;
    const int l = a.l, tid = threadIdx.x;
    constexpr bool in_lds = IN_LDS;
    double* W = stage_in(lds, a.H2, l, in_lds);
    bool ok = wg_chol_upper(W, l, l, &sflag);          // R2
    if (!ok) {
        if (tid == 0) *a.status |= DEV_NONFINITE;
        return;
    }
    // Z = R_P = R2 R1 (upper)
    for (int e = tid; e < l * l; e += SM_THREADS) {
        const int i = e % l, j = e / l;
        double s = 0.0;
        for (int k = i; k <= j; ++k) s += W[i + (size_t)k * l] * a.R1[k + (size_t)j * l];
        a.Z[e] = i <= j ? s : 0.0;
    }
    __syncthreads();
    // W = R_b^T with R_b = R_P R_Y^-1
    for (int e = tid; e < l * l; e += SM_THREADS) {
        const int i = e % l, j = e / l;
        double s = 0.0;
        for (int k = i; k <= j; ++k) s += a.Z[i + (size_t)k * l] * a.RYi[k + (size_t)j * l];
        W[j + (size_t)i * l] = i <= j ? s : 0.0;
    }
    __syncthreads();
    double* sig = in_lds ? lds_vecs(lds, l) : a.vec;
    double* nrm = sig + l;
    int* ord = in_lds ? (int*)(nrm + l) : a.ivec;
    int sw = wg_jacobi(W, l, l, l, sig, ord, nrm, a.max_sweeps, &sflag);
    if (tid == 0) {
        *a.sweeps = sw;
        if (sw > a.max_sweeps) *a.status |= DEV_NOCONV;
    }
    const int rk = a.K < l ? a.K : l;
    for (int e = tid; e < l * rk; e += SM_THREADS) {
        const int i = e % l, j = e / l;
        a.small_u[i + (size_t)j * l] = W[i + (size_t)ord[j] * l];
    }
    for (int j = tid; j < rk; j += SM_THREADS) a.s_out[j] = sig[ord[j]];
    __syncthreads();
    wg_sign_rule(a.small_u, l, rk, l, nullptr);
    // M2 = R_Y^-1 U~_rk
    for (int e = tid; e < l * rk; e += SM_THREADS) {
        const int i = e % l, j = e / l;
        double s = 0.0;
        for (int k = i; k < l; ++k) s += a.RYi[i + (size_t)k * l] * a.small_u[k + (size_t)j * l];
        a.M2[i + (size_t)j * l] = s;
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

// d[j] = ff * s[j]
__global__ void k_make_scale(double* d, const double* s, int r, double ff) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < r) d[j] = ff * s[j];
}

// ---------------------------------------------------------------------------
// APMOS small kernels.
// ---------------------------------------------------------------------------

// One work-group per partition: eigen-decomposition of G_i by one-sided
// Jacobi; W_i = V_i[:, :r] diag(sqrt(lambda_i[:r])) stored transposed.
template <bool IN_LDS>
__global__ __launch_bounds__(SM_THREADS) void k_apmos_local(ApmosLocalArgs a) {
    extern __shared__ double lds[];
    __shared__ int sflag;
    const int i = blockIdx.x, N = a.N, tid = threadIdx.x;
    constexpr bool in_lds = IN_LDS;
    double* G = stage_in(lds, a.G + (size_t)i * N * N, N, in_lds);
    double* sig = in_lds ? lds_vecs(lds, N) : a.vec + (size_t)i * 2 * N;
    double* nrm = sig + N;
    int* ord = in_lds ? (int*)(nrm + N) : a.ivec + (size_t)i * N;
    int sw = wg_jacobi(G, N, N, N, sig, ord, nrm, a.max_sweeps, &sflag);
    if (tid == 0 && sw > a.max_sweeps) atomicOr(a.status, (int)DEV_NOCONV);
    if (tid == 0) atomicMax(a.sweeps, sw);
    const int ldw = a.P * a.r;
    for (int e = tid; e < N * a.r; e += SM_THREADS) {
        int k = e % N, j = e / N;
        int src = ord[j];
        double lam = sig[src];
        double sj = sqrt(lam > 0.0 ? lam : 0.0);
        a.Wt[(size_t)(i * a.r + j) + (size_t)k * ldw] = G[k + (size_t)src * N] * sj;
    }
}


// W W^T = X Lambda^2 X^T by one-sided Jacobi; keep K; sign rule on X~;
// T = X~ diag(1 / Lambda~) with the guard Lambda~_K > N 2^-53 Lambda~_1.
template <bool IN_LDS>
__global__ __launch_bounds__(SM_THREADS) void k_apmos_global(ApmosGlobalArgs a) {
    extern __shared__ double lds[];
    __shared__ int sflag;
    const int N = a.N, tid = threadIdx.x;
    constexpr bool in_lds = IN_LDS;
    double* WW = stage_in(lds, a.WW, N, in_lds);
    double* sig = in_lds ? lds_vecs(lds, N) : a.vec;
    double* nrm = sig + N;
    int* ordv = in_lds ? (int*)(nrm + N) : a.ivec;
    int sw = wg_jacobi(WW, N, N, N, sig, ordv, nrm, a.max_sweeps, &sflag);
    if (tid == 0) {
        atomicMax(a.sweeps, sw);
        if (sw > a.max_sweeps) *a.status |= DEV_NOCONV;
    }
    for (int e = tid; e < N * a.K; e += SM_THREADS) {
        int k = e % N, j = e / N;
        a.X[k + (size_t)j * N] = WW[k + (size_t)ordv[j] * N];
    }
    for (int j = tid; j < a.K; j += SM_THREADS) {
        double lam = sig[ordv[j]];
        a.Lam[j] = sqrt(lam > 0.0 ? lam : 0.0);
    }
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
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (in_lds) hipLaunchKernelGGL(k_small_det1<true>, dim3(1), dim3(SM_THREADS), lds, st, a);
    else hipLaunchKernelGGL(k_small_det1<false>, dim3(1), dim3(SM_THREADS), lds, st, a);
    return hipGetLastError();
}
hipError_t launch_small_det2(const SmallArgs& a, hipStream_t st) {
    size_t lds = small_lds_bytes(a.n);
    const bool in_lds = (a.n) <= SM_LDS_MAX_N;
    const void* fn = in_lds ? (const void*)k_small_det2<true> : (const void*)k_small_det2<false>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (in_lds) hipLaunchKernelGGL(k_small_det2<true>, dim3(1), dim3(SM_THREADS), lds, st, a);
    else hipLaunchKernelGGL(k_small_det2<false>, dim3(1), dim3(SM_THREADS), lds, st, a);
    return hipGetLastError();
}
hipError_t launch_small_chol(const CholArgs& a, hipStream_t st) {
    size_t lds = small_lds_bytes(a.l);
    const bool in_lds = (a.l) <= SM_LDS_MAX_N;
    const void* fn = in_lds ? (const void*)k_small_chol<true> : (const void*)k_small_chol<false>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (in_lds) hipLaunchKernelGGL(k_small_chol<true>, dim3(1), dim3(256), lds, st, a);
    else hipLaunchKernelGGL(k_small_chol<false>, dim3(1), dim3(256), lds, st, a);
    return hipGetLastError();
}
hipError_t launch_small_rand_final(const RandFinalArgs& a, hipStream_t st) {
    size_t lds = small_lds_bytes(a.l);
    const bool in_lds = (a.l) <= SM_LDS_MAX_N;
    const void* fn = in_lds ? (const void*)k_small_rand_final<true> : (const void*)k_small_rand_final<false>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (in_lds) hipLaunchKernelGGL(k_small_rand_final<true>, dim3(1), dim3(SM_THREADS), lds, st, a);
    else hipLaunchKernelGGL(k_small_rand_final<false>, dim3(1), dim3(SM_THREADS), lds, st, a);
    return hipGetLastError();
}
hipError_t launch_scale_rows(double* X, int n, int m, int ldx, const double* d, int r, int times, hipStream_t st) {
    if (r <= 0 || n * m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_rows, dim3((n * m + 255) / 256), dim3(256), 0, st, X, n, m, ldx, d, r, times);
    return hipGetLastError();
}
hipError_t launch_make_scale(double* d, const double* s, int r, double ff, hipStream_t st) {
    if (r <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_make_scale, dim3((r + 255) / 256), dim3(256), 0, st, d, s, r, ff);
    return hipGetLastError();
}
hipError_t launch_apmos_local(const ApmosLocalArgs& a, hipStream_t st) {
    size_t lds = small_lds_bytes(a.N);
    const bool in_lds = (a.N) <= SM_LDS_MAX_N;
    const void* fn = in_lds ? (const void*)k_apmos_local<true> : (const void*)k_apmos_local<false>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (in_lds) hipLaunchKernelGGL(k_apmos_local<true>, dim3(a.P), dim3(SM_THREADS), lds, st, a);
    else hipLaunchKernelGGL(k_apmos_local<false>, dim3(a.P), dim3(SM_THREADS), lds, st, a);
    return hipGetLastError();
}
hipError_t launch_apmos_global(const ApmosGlobalArgs& a, hipStream_t st) {
    size_t lds = small_lds_bytes(a.N);
    const bool in_lds = (a.N) <= SM_LDS_MAX_N;
    const void* fn = in_lds ? (const void*)k_apmos_global<true> : (const void*)k_apmos_global<false>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (in_lds) hipLaunchKernelGGL(k_apmos_global<true>, dim3(1), dim3(SM_THREADS), lds, st, a);
    else hipLaunchKernelGGL(k_apmos_global<false>, dim3(1), dim3(SM_THREADS), lds, st, a);
    return hipGetLastError();
}

}  // namespace psvd
