// grad.hip -- small-core kernels of the reverse mode of the streaming SVD.
//
// One truncated-SVD step maps the panel C (M x n) to its leading rk left
// singular vectors and values.  With the full thin SVD C = U S V^T
// (U = C T_f, T_f = R^-1 U~ from the Cholesky-QR factor R = U~ S V^T) and
// cotangents U_bar (M x rk), s_bar (rk), the panel cotangent is
//   C_bar = U [diag(s_bar) + J S] V^T + (I - U U^T) U_bar S^-1 V^T,
//   J_ij = F_ij (H_ij - H_ji),  H = U^T U_bar,  F_ij = 1 / (s_j^2 - s_i^2),
// with U_bar and s_bar padded by zeros beyond rk (pairs with both indices
// >= rk carry nothing; F is set to 0 where |s_j^2 - s_i^2| <= 1e-12 s_1^2,
// the guard at near-degenerate pairs).  Written as two tall products:
//   C_bar = C Z1 + U_bar Z2,  Z1 = T_f (Inner - H S^-1) V^T,  Z2 = S_rk^-1 V_rk^T,
// so this kernel only forms the small matrices [D Z1; Z2].
#include "kernels.h"

namespace psvd {

constexpr int GR_THREADS = 1024;

__device__ void grad_trsm_upper(const double* R, int n, const double* B, double* X) {
    // X = R^-1 B (n x n), row by row from the bottom, all columns in parallel.
    for (int i = n - 1; i >= 0; --i) {
        const double rii = R[i + (size_t)i * n];
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            double s = B[i + (size_t)j * n];
            for (int k = i + 1; k < n; ++k) s -= R[i + (size_t)k * n] * X[k + (size_t)j * n];
            X[i + (size_t)j * n] = s / rii;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(GR_THREADS) void k_grad_core(GradCoreArgs a) {
    extern __shared__ double lds[];
    const int n = a.n, rk = a.rk, r = a.r, tid = threadIdx.x;
    const double* R = a.R;
    const double* Ut = a.Ut;
    const double* S = a.S;
    if (*a.status & (DEV_FALLBACK | DEV_NONFINITE | DEV_BREAKDOWN | DEV_NOCONV)) return;
    // T_f = R^-1 U~ with R and the solution in LDS when they fit.
    const bool in_lds = 2 * (size_t)n * n * sizeof(double) <= 150 * 1024;
    if (in_lds) {
        double* Rl = lds;
        double* Xl = lds + (size_t)n * n;
        for (int e = tid; e < n * n; e += GR_THREADS) Rl[e] = R[e];
        __syncthreads();
        grad_trsm_upper(Rl, n, Ut, Xl);
        for (int e = tid; e < n * n; e += GR_THREADS) a.Tf[e] = Xl[e];
    } else {
        grad_trsm_upper(R, n, Ut, a.Tf);
    }
    __syncthreads();
    // V = R^T U~ S^-1
    for (int e = tid; e < n * n; e += GR_THREADS) {
        int i = e % n, j = e / n;
        double s = 0.0;
        for (int k = 0; k <= i; ++k) s += R[k + (size_t)i * n] * Ut[k + (size_t)j * n];
        a.V[e] = S[j] > 0.0 ? s / S[j] : 0.0;
    }
    __syncthreads();
    // H = T_f^T E (n x rk), E = C^T U_bar
    for (int e = tid; e < n * rk; e += GR_THREADS) {
        int i = e % n, j = e / n;
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += a.Tf[k + (size_t)i * n] * a.E[k + (size_t)j * n];
        a.H[e] = s;
    }
    __syncthreads();
    // W1 = (Inner - H S^-1) with Inner = diag(s_bar) + J S  (n x n), stored in Wk
    const double s1sq = S[0] * S[0];
    for (int e = tid; e < n * n; e += GR_THREADS) {
        int i = e % n, j = e / n;
        double v = 0.0;
        if (i == j) {
            v = j < rk ? a.sbar[j] : 0.0;
        } else if (i < rk || j < rk) {
            double hij = j < rk ? a.H[i + (size_t)j * n] : 0.0;
            double hji = i < rk ? a.H[j + (size_t)i * n] : 0.0;
            double den = S[j] * S[j] - S[i] * S[i];
            double f = fabs(den) > 1e-12 * s1sq ? 1.0 / den : 0.0;
            v = f * (hij - hji) * S[j];
        }
        if (j < rk && S[j] > 0.0) v -= a.H[i + (size_t)j * n] / S[j];
        a.Wk[e] = v;
    }
    __syncthreads();
    // W2 = W1 V^T  -> reuse H storage is too small; write into Z (n x n) temporarily
    for (int e = tid; e < n * n; e += GR_THREADS) {
        int i = e % n, j = e / n;
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += a.Wk[i + (size_t)k * n] * a.V[j + (size_t)k * n];
        a.Zt[e] = s;
    }
    __syncthreads();
    // Z1 = T_f W2 ; rows of the C' part scaled by D; output column c < r scaled by d[c].
    const int ldz = n + rk;
    for (int e = tid; e < n * n; e += GR_THREADS) {
        int i = e % n, c = e / n;
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += a.Tf[i + (size_t)k * n] * a.Zt[k + (size_t)c * n];
        if (i < r) s *= a.d[i];
        if (c < r) a.Zu[i + (size_t)c * ldz] = s * a.d[c];
        else a.Za[i + (size_t)(c - r) * ldz] = s;
    }
    // Z2 = S_rk^-1 V_rk^T  (rows n .. n + rk - 1)
    for (int e = tid; e < rk * n; e += GR_THREADS) {
        int j = e % rk, c = e / rk;
        double s = S[j] > 0.0 ? a.V[c + (size_t)j * n] / S[j] : 0.0;
        if (c < r) a.Zu[(n + j) + (size_t)c * ldz] = s * a.d[c];
        else a.Za[(n + j) + (size_t)(c - r) * ldz] = s;
    }
}

// s_bar_prev[c] = (U_prev^T U_bar_new)_cc / s_prev[c]  (0 where s_prev[c] = 0).
__global__ void k_grad_sbar(const double* G, int r, const double* s_prev, double* sbar) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < r) sbar[c] = s_prev[c] > 0.0 ? G[c + (size_t)c * r] / s_prev[c] : 0.0;
}

hipError_t launch_grad_core(const GradCoreArgs& a, hipStream_t st) {
    size_t lds = 2 * (size_t)a.n * a.n * sizeof(double);
    if (lds > 150 * 1024) lds = 64;
    hipError_t e = hipFuncSetAttribute((const void*)k_grad_core, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad_core, dim3(1), dim3(GR_THREADS), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_grad_sbar(const double* G, int r, const double* s_prev, double* sbar, hipStream_t st) {
    if (r <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_sbar, dim3((r + 255) / 256), dim3(256), 0, st, G, r, s_prev, sbar);
    return hipGetLastError();
}

}  // namespace psvd
