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
__device__ bool wg_chol_upper(double* A, int n, int lda, int* sflag) {
    const int tid = threadIdx.x;
    if (tid == 0) *sflag = 0;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (tid == 0) {
            double d = A[k + (size_t)k * lda];
            if (!(d > 0.0) || !finite_d(d)) *sflag = 1;
            else A[k + (size_t)k * lda] = sqrt(d);
        }
        __syncthreads();
        if (*sflag) return false;
        const double rkk = A[k + (size_t)k * lda];
        for (int j = k + 1 + tid; j < n; j += SM_THREADS) A[k + (size_t)j * lda] /= rkk;
        __syncthreads();
        // trailing update of the upper triangle: A[i][j] -= R[k][i] R[k][j], k < i <= j
        const int m = n - k - 1;
        const int tot = m * (m + 1) / 2;
        for (int e = tid; e < tot; e += SM_THREADS) {
            // map e -> (i, j) with i <= j in the trailing block (column-wise packing)
            int jj = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
            while ((jj + 1) * (jj + 2) / 2 <= e) ++jj;
            while (jj * (jj + 1) / 2 > e) --jj;
            int ii = e - jj * (jj + 1) / 2;
            int i = k + 1 + ii, j = k + 1 + jj;
            A[i + (size_t)j * lda] -= A[k + (size_t)i * lda] * A[k + (size_t)j * lda];
        }
        __syncthreads();
    }
    // zero the strict lower triangle
    for (int e = tid; e < n * n; e += SM_THREADS) {
        int i = e % n, j = e / n;
        if (i > j) A[i + (size_t)j * lda] = 0.0;
    }
    __syncthreads();
    return true;
}

// Ri = R^-1 for upper triangular R (n x n): column j solves R x = e_j.
__device__ void wg_trinv_upper(const double* R, int n, int ldr, double* Ri, int ldi) {
    const int tid = threadIdx.x;
    for (int j = tid; j < n; j += SM_THREADS) {
        double* x = Ri + (size_t)j * ldi;
        for (int i = n - 1; i >= 0; --i) {
            if (i > j) {
                x[i] = 0.0;
                continue;
            }
            double s = (i == j) ? 1.0 : 0.0;
            for (int k = i + 1; k <= j; ++k) s -= R[i + (size_t)k * ldr] * x[k];
            x[i] = s / R[i + (size_t)i * ldr];
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
// One-sided Jacobi on the columns of Z (m x n, ldz), in place.  On return
// the columns are mutually orthogonal to the tolerance m * 2^-53; sig[j] =
// ||z_j|| and z_j /= sig[j] (0 columns stay 0).  order[0..n) lists the
// columns by descending sig (stable).  Parallel round-robin ordering: each
// round rotates n/2 disjoint pairs, one pair per wave at a time.
// Returns the number of sweeps (> max_sweeps: not converged).
// ---------------------------------------------------------------------------
__device__ int wg_jacobi(double* Z, int m, int n, int ldz, double* sig, int* order, double* nrm, int max_sweeps,
                         int* sflag) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const double tol = (double)m * 0x1p-53;
    const int ne = n + (n & 1);
    int sweep = 0;
    for (;;) {
        // exact column norms at the start of every sweep
        for (int j = w; j < n; j += SM_WAVES) {
            const double* z = Z + (size_t)j * ldz;
            double s = 0.0;
            for (int i = lane; i < m; i += 64) s += z[i] * z[i];
            s = wave_sum(s);
            if (lane == 0) nrm[j] = s;
        }
        if (tid == 0) *sflag = 0;
        __syncthreads();
        // columns below (m u)^2 of the largest carry only rounding noise: they
        // are not rotated (they cannot be made more orthogonal).
        double nmax = 0.0;
        for (int j = 0; j < n; ++j) nmax = fmax(nmax, nrm[j]);
        const double negl = nmax * tol * tol;
        if (sweep >= max_sweeps) {
            ++sweep;
            break;
        }
        for (int t = 0; t < ne - 1; ++t) {
            for (int pi = w; pi < ne / 2; pi += SM_WAVES) {
                int pa = pi, pb = ne - 1 - pi;
                int ca = pa == 0 ? 0 : 1 + (pa - 1 + t) % (ne - 1);
                int cb = pb == 0 ? 0 : 1 + (pb - 1 + t) % (ne - 1);
                int p = ca < cb ? ca : cb, q = ca < cb ? cb : ca;
                if (q >= n) continue;
                double* zp = Z + (size_t)p * ldz;
                double* zq = Z + (size_t)q * ldz;
                double g = 0.0;
                for (int i = lane; i < m; i += 64) g += zp[i] * zq[i];
                g = wave_sum(g);
                double al = nrm[p], be = nrm[q];
                if (!(al > negl) || !(be > negl)) continue;
                if (fabs(g) <= tol * sqrt(al) * sqrt(be)) continue;
                double zeta = (be - al) / (2.0 * g);
                double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
                for (int i = lane; i < m; i += 64) {
                    double a = zp[i], b = zq[i];
                    zp[i] = c * a - s * b;
                    zq[i] = s * a + c * b;
                }
                if (lane == 0) {
                    nrm[p] = al - tt * g;
                    nrm[q] = be + tt * g;
                    *sflag = 1;
                }
            }
            __syncthreads();
        }
        ++sweep;
        int rotated = *sflag;
        __syncthreads();
        if (!rotated) break;
    }
    // singular values, normalisation
    for (int j = w; j < n; j += SM_WAVES) {
        double* z = Z + (size_t)j * ldz;
        double s = 0.0;
        for (int i = lane; i < m; i += 64) s += z[i] * z[i];
        s = sqrt(wave_sum(s));
        for (int i = lane; i < m; i += 64) z[i] = s > 0.0 ? z[i] / s : 0.0;
        if (lane == 0) sig[j] = s;
    }
    __syncthreads();
    // stable descending order
    for (int j = tid; j < n; j += SM_THREADS) {
        double sj = sig[j];
        int rank = 0;
        for (int i = 0; i < n; ++i) {
            double si = sig[i];
            if (si > sj || (si == sj && i < j)) ++rank;
        }
        order[rank] = j;
    }
    __syncthreads();
    return sweep;
}

// Sign rule: column j of X (rows x k) gets its largest-magnitude entry
// (lowest index on ties) non-negative; flips recorded in flip[j].
__device__ void wg_sign_rule(double* X, int rows, int k, int ldx, double* flip) {
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

__device__ __forceinline__ double dscale(const SmallArgs& a, int j) { return j < a.r ? a.d[j] : 1.0; }

__global__ __launch_bounds__(SM_THREADS) void k_small_det1(SmallArgs a) {
    __shared__ int sflag;
    const int n = a.n, tid = threadIdx.x;
    // G <- D G' D, NaN/Inf check
    __shared__ int nonfinite;
    if (tid == 0) nonfinite = 0;
    __syncthreads();
    for (int e = tid; e < n * n; e += SM_THREADS) {
        int i = e % n, j = e / n;
        double v = a.G[e] * dscale(a, i) * dscale(a, j);
        if (!finite_d(v)) nonfinite = 1;
        a.G[e] = v;
        a.R1[e] = v;
    }
    __syncthreads();
    if (nonfinite) {
        if (tid == 0) *a.status |= DEV_NONFINITE;
        return;
    }
    bool ok = wg_chol_upper(a.R1, n, n, &sflag);
    if (ok) {
        wg_trinv_upper(a.R1, n, n, a.Ri, n);
        // Xn = D R1^-1
        for (int e = tid; e < n * n; e += SM_THREADS) {
            int i = e % n;
            a.Xn[e] = a.Ri[e] * dscale(a, i);
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
    for (int e = tid; e < n * n; e += SM_THREADS) a.Z[e] = a.G[e];
    __syncthreads();
    double* sig = a.vec;
    double* nrm = a.vec + n;
    int sw = wg_jacobi(a.Z, n, n, n, sig, a.ivec, nrm, a.max_sweeps, &sflag);
    if (tid == 0) {
        *a.sweeps = sw;
        if (sw > a.max_sweeps) *a.status |= DEV_NOCONV;
    }
    const int rk = a.K < n ? a.K : n;
    // sorted eigenvectors (normalised columns of Z) -> small_u, sign rule
    for (int e = tid; e < n * rk; e += SM_THREADS) {
        int i = e % n, j = e / n;
        a.small_u[i + (size_t)j * n] = a.Z[i + (size_t)a.ivec[j] * n];
    }
    __syncthreads();
    wg_sign_rule(a.small_u, n, rk, n, nullptr);
    for (int j = tid; j < rk; j += SM_THREADS) {
        double lam = sig[a.ivec[j]];
        a.s_out[j] = sqrt(lam > 0.0 ? lam : 0.0);
    }
    __syncthreads();
    for (int e = tid; e < n * rk; e += SM_THREADS) {
        int i = e % n, j = e / n;
        double sj = a.s_out[j];
        a.T[i + (size_t)j * n] = sj > 0.0 ? dscale(a, i) * a.small_u[i + (size_t)j * n] / sj : 0.0;
    }
}

// After the second Gram G2 = Q1^T Q1: R2 = chol(G2), R = R2 R1, Jacobi SVD of
// R -> U~ (left vectors), S; sort, sign rule, keep rk = min(K, n);
// T = D R^-1 U~_rk.
__global__ __launch_bounds__(SM_THREADS) void k_small_det2(SmallArgs a) {
    __shared__ int sflag;
    if (*a.status & (DEV_FALLBACK | DEV_NONFINITE | DEV_BREAKDOWN)) return;
    const int n = a.n, tid = threadIdx.x;
    bool ok = wg_chol_upper(a.G2, n, n, &sflag);
    if (!ok) {
        // Q1 is orthonormal to working accuracy once the first factor exists;
        // a breakdown here means non-finite data.
        if (tid == 0) *a.status |= DEV_NONFINITE;
        return;
    }
    // R = R2 R1 (upper) -> Z
    for (int e = tid; e < n * n; e += SM_THREADS) {
        int i = e % n, j = e / n;
        double s = 0.0;
        for (int k = i; k <= j; ++k) s += a.G2[i + (size_t)k * n] * a.R1[k + (size_t)j * n];
        a.Z[e] = (i <= j) ? s : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += SM_THREADS) a.G[e] = a.Z[e];  // keep R
    __syncthreads();
    double* sig = a.vec;
    double* nrm = a.vec + n;
    int sw = wg_jacobi(a.Z, n, n, n, sig, a.ivec, nrm, a.max_sweeps, &sflag);
    if (tid == 0) {
        *a.sweeps = sw;
        if (sw > a.max_sweeps) *a.status |= DEV_NOCONV;
    }
    const int rk = a.K < n ? a.K : n;
    for (int e = tid; e < n * rk; e += SM_THREADS) {
        int i = e % n, j = e / n;
        a.small_u[i + (size_t)j * n] = a.Z[i + (size_t)a.ivec[j] * n];
    }
    for (int j = tid; j < rk; j += SM_THREADS) a.s_out[j] = sig[a.ivec[j]];
    __syncthreads();
    wg_sign_rule(a.small_u, n, rk, n, nullptr);
    // The lift reads Q1 = C D R1^-1 (the first Cholesky-QR factor, kept by the
    // second Gram pass): U = Q1 R2^-1 U~_rk, so T = R2^-1 U~ (back substitution).
    const double* R2 = a.G2;
    for (int j = tid; j < rk; j += SM_THREADS) {
        double* x = a.T + (size_t)j * n;
        const double* u = a.small_u + (size_t)j * n;
        for (int i = n - 1; i >= 0; --i) {
            double s = u[i];
            for (int k = i + 1; k < n; ++k) s -= R2[i + (size_t)k * n] * x[k];
            x[i] = s / R2[i + (size_t)i * n];
        }
    }
}

// ---------------------------------------------------------------------------
// Randomized-path small kernels.
// ---------------------------------------------------------------------------

// R = chol(H) in place, Ri = R^-1.  On breakdown a diagonal shift
// s = 11 (l^2 + l) 2^-53 ||H||_F (shifted Cholesky-QR of Fukaya et al. 2020)
// is added and the factorisation repeated.
__global__ __launch_bounds__(SM_THREADS) void k_small_chol(CholArgs a) {
    __shared__ int sflag;
    __shared__ double fro;
    const int l = a.l, tid = threadIdx.x;
    if (*a.status & (DEV_NONFINITE | DEV_BREAKDOWN)) return;
    if (tid == 0) fro = 0.0;
    __syncthreads();
    // Keep a copy of H in Ri for the retry.
    for (int e = tid; e < l * l; e += SM_THREADS) a.Ri[e] = a.H[e];
    __syncthreads();
    bool ok = wg_chol_upper(a.H, l, l, &sflag);
    if (!ok) {
        if (tid == 0) {
            double f = 0.0;
            for (int e = 0; e < l * l; ++e) f += a.Ri[e] * a.Ri[e];
            fro = sqrt(f);
            *a.status |= a.flag_bit;
        }
        __syncthreads();
        double shift = 11.0 * ((double)l * l + l) * 0x1p-53 * fro;
        for (int e = tid; e < l * l; e += SM_THREADS) {
            int i = e % l, j = e / l;
            a.H[e] = a.Ri[e] + (i == j ? shift : 0.0);
        }
        __syncthreads();
        ok = wg_chol_upper(a.H, l, l, &sflag);
        if (!ok) {
            if (tid == 0) *a.status |= DEV_NONFINITE;
            return;
        }
    }
    wg_trinv_upper(a.H, l, l, a.Ri, l);
}


// R_P = chol(H2) R1 (QR factor of P); R_b = R_P R_Y^-1; the left singular
// vectors of B = R_Y^-T P^T are those of R_b^T: one-sided Jacobi on R_b^T.
__global__ __launch_bounds__(SM_THREADS) void k_small_rand_final(RandFinalArgs a) {
    __shared__ int sflag;
    if (*a.status & (DEV_NONFINITE | DEV_BREAKDOWN)) return;
    const int l = a.l, tid = threadIdx.x;
    bool ok = wg_chol_upper(a.H2, l, l, &sflag);
    if (!ok) {
        if (tid == 0) *a.status |= DEV_NONFINITE;
        return;
    }
    // M2 <- R_P = R2 R1 (upper), temporarily
    for (int e = tid; e < l * l; e += SM_THREADS) {
        int i = e % l, j = e / l;
        double s = 0.0;
        for (int k = i; k <= j; ++k) s += a.H2[i + (size_t)k * l] * a.R1[k + (size_t)j * l];
        a.Z[e] = i <= j ? s : 0.0;
    }
    __syncthreads();
    // R_b = R_P R_Y^-1 ; Z <- R_b^T
    for (int e = tid; e < l * l; e += SM_THREADS) {
        int i = e % l, j = e / l;
        double s = 0.0;
        for (int k = i; k <= j; ++k) s += a.Z[i + (size_t)k * l] * a.RYi[k + (size_t)j * l];
        a.H2[j + (size_t)i * l] = i <= j ? s : 0.0;   // transpose into H2
    }
    __syncthreads();
    double* sig = a.vec;
    double* nrm = a.vec + l;
    int sw = wg_jacobi(a.H2, l, l, l, sig, a.ivec, nrm, a.max_sweeps, &sflag);
    if (tid == 0) {
        *a.sweeps = sw;
        if (sw > a.max_sweeps) *a.status |= DEV_NOCONV;
    }
    const int rk = a.K < l ? a.K : l;
    for (int e = tid; e < l * rk; e += SM_THREADS) {
        int i = e % l, j = e / l;
        a.small_u[i + (size_t)j * l] = a.H2[i + (size_t)a.ivec[j] * l];
    }
    for (int j = tid; j < rk; j += SM_THREADS) a.s_out[j] = sig[a.ivec[j]];
    __syncthreads();
    wg_sign_rule(a.small_u, l, rk, l, nullptr);
    // M2 = R_Y^-1 U~_rk
    for (int e = tid; e < l * rk; e += SM_THREADS) {
        int i = e % l, j = e / l;
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
__global__ __launch_bounds__(SM_THREADS) void k_apmos_local(ApmosLocalArgs a) {
    __shared__ int sflag;
    const int i = blockIdx.x, N = a.N, tid = threadIdx.x;
    double* G = a.G + (size_t)i * N * N;
    double* sig = a.vec + (size_t)i * 2 * N;
    double* nrm = sig + N;
    int* ord = a.ivec + (size_t)i * N;
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
__global__ __launch_bounds__(SM_THREADS) void k_apmos_global(ApmosGlobalArgs a) {
    __shared__ int sflag;
    const int N = a.N, tid = threadIdx.x;
    double* sig = a.vec;
    double* nrm = a.vec + N;
    int sw = wg_jacobi(a.WW, N, N, N, sig, a.ivec, nrm, a.max_sweeps, &sflag);
    if (tid == 0) {
        atomicMax(a.sweeps, sw);
        if (sw > a.max_sweeps) *a.status |= DEV_NOCONV;
    }
    for (int e = tid; e < N * a.K; e += SM_THREADS) {
        int k = e % N, j = e / N;
        a.X[k + (size_t)j * N] = a.WW[k + (size_t)a.ivec[j] * N];
    }
    for (int j = tid; j < a.K; j += SM_THREADS) {
        double lam = sig[a.ivec[j]];
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
    hipLaunchKernelGGL(k_small_det1, dim3(1), dim3(SM_THREADS), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_small_det2(const SmallArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_small_det2, dim3(1), dim3(SM_THREADS), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_small_chol(const CholArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_small_chol, dim3(1), dim3(SM_THREADS), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_small_rand_final(const RandFinalArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_small_rand_final, dim3(1), dim3(SM_THREADS), 0, st, a);
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
    hipLaunchKernelGGL(k_apmos_local, dim3(a.P), dim3(SM_THREADS), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_apmos_global(const ApmosGlobalArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_apmos_global, dim3(1), dim3(SM_THREADS), 0, st, a);
    return hipGetLastError();
}

}  // namespace psvd
