/*
 * psvd_oracle.c -- plain, slow, FP64 CPU oracle for the streaming / randomized /
 * partitioned SVD of Maulik & Mengaldo, "PyParSVD" (arXiv 2108.08845).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the GPU path.
 *
 * Everything is double precision, column-major (element (i,j) of a matrix
 * with leading dimension ld sits at a[i + j*ld]), no BLAS and no LAPACK.
 * Each routine follows the mathematical definition or the algorithm in the
 * paper's order; OpenMP only splits independent loop iterations, and every
 * reduction over a long dimension is summed in a fixed chunk order so the
 * result does not depend on the thread count.
 *
 * Routines and the passages they follow:
 *   orc_philox4x32_10 / orc_omega  -- Gaussian test matrix of Sec. 3.3 (the
 *       paper draws it from a zero-mean unit-variance normal for every
 *       randomized SVD).  Counter-based generator: Philox4x32-10 of Salmon,
 *       Moraes, Dror & Shaw (SC'11); normals by Box & Muller (1958).
 *   orc_hhqr         -- thin Householder QR (Golub & Van Loan, Alg. 5.2.1),
 *       the QR decomposition of Algorithm 1 (initialisation and update).
 *   orc_jacobi_svd   -- one-sided cyclic Jacobi SVD (Hestenes 1958), the
 *       SVD of the R factor in Algorithm 1, and Eq. (9).
 *   orc_stream_update -- one batch of Algorithm 1 (Sec. 3.1): deterministic
 *       (QR of [ff*U*D | A], SVD of R, keep K) or, with a test matrix,
 *       the randomized range finder of Eqs. (7)-(11) applied to the same
 *       panel (power iterations per Halko, Martinsson & Tropp 2011, Alg. 4.4).
 *   orc_apmos        -- Algorithm 2 / Eqs. (3)-(6) (Sec. 3.2) on P partitions.
 *   orc_low_rank_svd -- the low-rank SVD of Eqs. (7)-(11) applied to a small
 *       matrix, where the parallel variant of Sec. 3 randomizes: the SVD of
 *       W in Algorithm 2 (orc_apmos_lr) and of the combined R factor of the
 *       partitioned update (orc_pstream_update_lr).
 *   orc_stream_grad  -- reverse-mode derivative of the loss
 *       ||A - U U^T A||_F^2 + sum_j w_j s_j through the deterministic
 *       streaming recursion (adjoint of the thin SVD; the paper is silent).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-4)
#define ORC_ENOCONV (-6)

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. 2011).                                       */
/* ------------------------------------------------------------------------ */

static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t o0 = hi1 ^ c[1] ^ k[0];
    uint32_t o2 = hi0 ^ c[3] ^ k[1];
    c[0] = o0;
    c[1] = lo1;
    c[2] = o2;
    c[3] = lo0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

/* Round a float to the nearest bfloat16 (ties to even); returns the value. */
static double round_bf16_from_float(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) { /* inf or nan: keep */
        if (u & 0x007FFFFFu) u |= 0x00400000u;
        u &= 0xFFFF0000u;
    } else {
        uint32_t lsb = (u >> 16) & 1u;
        u += 0x7FFFu + lsb;
        u &= 0xFFFF0000u;
    }
    float g;
    memcpy(&g, &u, 4);
    return (double)g;
}

/*
 * Gaussian test matrix Omega (n x ell, column-major) for batch `batch`.
 * Element e = i + j*n.  Philox call t (counter = (t_lo, t_hi, batch_lo,
 * batch_hi), key = (seed_lo, seed_hi)) gives x0..x3; two 53-bit uniforms
 *   u1 = ((x0>>5)*2^26 + (x1>>6)) * 2^-53,  u2 likewise from (x2, x3),
 * and Box-Muller gives
 *   z0 = sqrt(-2 ln(1-u1)) cos(2 pi u2)   -> element 2t
 *   z1 = sqrt(-2 ln(1-u1)) sin(2 pi u2)   -> element 2t+1,
 * with log, cos and sin from the C library, each by its own call.
 * precision 0 keeps the double, 1 rounds to float (RNE), 2 rounds to float
 * and then to bfloat16 (both RNE).
 */
void orc_omega(uint64_t seed, int64_t batch, int64_t n, int64_t ell, int precision, double* out)
{
    const int64_t total = n * ell;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t t = 0; 2 * t < total; ++t) {
        uint32_t ctr[4] = {(uint32_t)t, (uint32_t)((uint64_t)t >> 32), (uint32_t)batch,
                           (uint32_t)((uint64_t)batch >> 32)};
        uint32_t x[4];
        orc_philox4x32_10(ctr, key, x);
        double u1 = ((double)(x[0] >> 5) * 67108864.0 + (double)(x[1] >> 6)) * (1.0 / 9007199254740992.0);
        double u2 = ((double)(x[2] >> 5) * 67108864.0 + (double)(x[3] >> 6)) * (1.0 / 9007199254740992.0);
        double rad = sqrt(-2.0 * log(1.0 - u1));
        /* cos and sin each by its own libm call (a volatile argument keeps the
           compiler from merging them into sincos, whose last bit may differ). */
        volatile double ang = two_pi * u2;
        double z[2] = {rad * cos(ang), rad * sin(ang)};
        for (int h = 0; h < 2; ++h) {
            int64_t e = 2 * t + h;
            if (e >= total) break;
            double v = z[h];
            if (precision == 1) v = (double)(float)v;
            else if (precision == 2) v = round_bf16_from_float((float)v);
            out[e] = v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Dense helpers (plain loops).                                             */
/* ------------------------------------------------------------------------ */

/* Dot product with four interleaved partial sums, combined in a fixed order. */
static double dot(const double* a, const double* b, int64_t len)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t i = 0;
    for (; i + 4 <= len; i += 4) {
        s0 += a[i] * b[i];
        s1 += a[i + 1] * b[i + 1];
        s2 += a[i + 2] * b[i + 2];
        s3 += a[i + 3] * b[i + 3];
    }
    for (; i < len; ++i) s0 += a[i] * b[i];
    return (s0 + s1) + (s2 + s3);
}

/* C (m x n, ldc) = A (m x k, lda) * B (k x n, ldb). Rows split across threads. */
static void mm_nn(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, const double* B,
                  int64_t ldb, double* C, int64_t ldc)
{
    const int64_t rb = 256;
    const int64_t nblk = (m + rb - 1) / rb;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nblk; ++b) {
        int64_t i0 = b * rb, i1 = i0 + rb < m ? i0 + rb : m;
        for (int64_t j = 0; j < n; ++j) {
            double* c = C + IDX(0, j, ldc);
            for (int64_t i = i0; i < i1; ++i) c[i] = 0.0;
            for (int64_t p = 0; p < k; ++p) {
                double bv = B[IDX(p, j, ldb)];
                const double* a = A + IDX(0, p, lda);
                for (int64_t i = i0; i < i1; ++i) c[i] += a[i] * bv;
            }
        }
    }
}

/*
 * C (m x n, ldc) = A^T (A: k x m, lda) * B (k x n, ldb), a reduction over the
 * long dimension k.  Partial products over fixed chunks of k are summed in
 * chunk order (independent of the number of threads).
 */
static int mm_tn(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, const double* B,
                 int64_t ldb, double* C, int64_t ldc)
{
    int64_t chunk = 8192;
    if (k / chunk > 512) chunk = (k + 511) / 512;
    const int64_t nch = k > 0 ? (k + chunk - 1) / chunk : 0;
    double* part = NULL;
    if (nch > 1) {
        part = (double*)calloc((size_t)nch * (size_t)(m * n), sizeof(double));
        if (!part) return ORC_ENOMEM;
    }
#pragma omp parallel for schedule(dynamic)
    for (int64_t c = 0; c < nch; ++c) {
        int64_t p0 = c * chunk, p1 = p0 + chunk < k ? p0 + chunk : k;
        for (int64_t j = 0; j < n; ++j) {
            const double* b = B + IDX(0, j, ldb);
            for (int64_t i = 0; i < m; ++i) {
                const double* a = A + IDX(0, i, lda);
                double acc = dot(a + p0, b + p0, p1 - p0);
                if (nch > 1) part[(size_t)c * (size_t)(m * n) + (size_t)(i + j * m)] = acc;
                else C[IDX(i, j, ldc)] = acc;
            }
        }
    }
    if (nch > 1) {
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i) {
                double acc = 0.0;
                for (int64_t c = 0; c < nch; ++c) acc += part[(size_t)c * (size_t)(m * n) + (size_t)(i + j * m)];
                C[IDX(i, j, ldc)] = acc;
            }
        free(part);
    } else if (nch == 0) {
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i) C[IDX(i, j, ldc)] = 0.0;
    }
    return ORC_OK;
}

/* Sum of squares of x[0..len) in fixed chunk order. */
static double sumsq(const double* x, int64_t len)
{
    double tot = 0.0;
    const int64_t chunk = 65536;
    for (int64_t c0 = 0; c0 < len; c0 += chunk) {
        int64_t c1 = c0 + chunk < len ? c0 + chunk : len;
        tot += dot(x + c0, x + c0, c1 - c0);
    }
    return tot;
}

/* ------------------------------------------------------------------------ */
/* Householder thin QR (Golub & Van Loan, Alg. 5.2.1).                      */
/* ------------------------------------------------------------------------ */

/*
 * A (m x n, lda), m >= n.  Writes Q (m x n, ld m) with orthonormal columns
 * and R (n x n, ld n) upper triangular with R_jj >= 0, A = Q R.
 * Each reflector H_k = I - tau v v^T (v_k = 1) maps A[k:,k] to beta e_1 with
 * beta = -sign(alpha) ||x|| (no cancellation); the signs of row j of R and
 * column j of Q are flipped afterwards wherever R_jj < 0.
 */
int orc_hhqr(int64_t m, int64_t n, const double* A, int64_t lda, double* Q, double* R)
{
    if (m < n || n < 0) return ORC_EINVAL;
    double* W = (double*)malloc((size_t)m * (size_t)(n > 0 ? n : 1) * sizeof(double));
    double* tau = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!W || !tau) {
        free(W);
        free(tau);
        return ORC_ENOMEM;
    }
    for (int64_t j = 0; j < n; ++j) memcpy(W + IDX(0, j, m), A + IDX(0, j, lda), (size_t)m * sizeof(double));

    for (int64_t k = 0; k < n; ++k) {
        double* x = W + IDX(k, k, m);
        int64_t len = m - k;
        double alpha = x[0];
        double nrm = sqrt(sumsq(x, len));
        if (nrm == 0.0) {
            tau[k] = 0.0;
            continue;
        }
        double beta = alpha >= 0.0 ? -nrm : nrm;
        double v0 = alpha - beta;
        tau[k] = (beta - alpha) / beta;
        for (int64_t i = 1; i < len; ++i) x[i] /= v0;
        x[0] = beta; /* R_kk; v_0 = 1 implicitly */
        const double tk = tau[k];
#pragma omp parallel for schedule(static)
        for (int64_t j = k + 1; j < n; ++j) {
            double* a = W + IDX(k, j, m);
            double d = a[0] + dot(x + 1, a + 1, len - 1);
            d *= tk;
            a[0] -= d;
            for (int64_t i = 1; i < len; ++i) a[i] -= d * x[i];
        }
    }
    /* R */
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) R[IDX(i, j, n)] = i <= j ? W[IDX(i, j, m)] : 0.0;
    /* Q = H_0 ... H_{n-1} [I; 0], accumulated backwards. */
    for (int64_t j = 0; j < n; ++j) {
        double* qj = Q + IDX(0, j, m);
        memset(qj, 0, (size_t)m * sizeof(double));
        qj[j] = 1.0;
    }
    for (int64_t k = n - 1; k >= 0; --k) {
        const double tk = tau[k];
        if (tk == 0.0) continue;
        const double* v = W + IDX(k, k, m); /* v[0] = 1 implicitly */
        int64_t len = m - k;
#pragma omp parallel for schedule(static)
        for (int64_t j = k; j < n; ++j) {
            double* a = Q + IDX(k, j, m);
            double d = a[0] + dot(v + 1, a + 1, len - 1);
            d *= tk;
            a[0] -= d;
            for (int64_t i = 1; i < len; ++i) a[i] -= d * v[i];
        }
    }
    /* Non-negative diagonal of R. */
    for (int64_t j = 0; j < n; ++j) {
        if (R[IDX(j, j, n)] < 0.0) {
            for (int64_t c = j; c < n; ++c) R[IDX(j, c, n)] = -R[IDX(j, c, n)];
            double* qj = Q + IDX(0, j, m);
            for (int64_t i = 0; i < m; ++i) qj[i] = -qj[i];
        }
    }
    free(W);
    free(tau);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* One-sided Jacobi SVD (Hestenes 1958), cyclic-by-rows ordering.           */
/* ------------------------------------------------------------------------ */


/*
 * A (m x n, lda), m >= n.  Computes A = U diag(s) V^T with U (m x n, ld m),
 * s (n) descending (stable: equal values keep their column order) and
 * V (n x n, ld n).  Either U or V may be NULL.  A pair (p, q) is rotated
 * while |a_p^T a_q| > m * 2^-53 * ||a_p|| ||a_q||; the rotation angle comes
 * from zeta = (beta - alpha) / (2 gamma), t = sign(zeta) / (|zeta| +
 * sqrt(1 + zeta^2)).  Columns with s_j = 0 leave U[:, j] = 0.
 * Returns ORC_ENOCONV if max_sweeps sweeps do not converge.
 */
int orc_jacobi_svd(int64_t m, int64_t n, const double* A, int64_t lda, double* U, double* s, double* V,
                   int max_sweeps, int* sweeps_out)
{
    if (m < n || n < 0) return ORC_EINVAL;
    double* W = (double*)malloc((size_t)m * (size_t)(n > 0 ? n : 1) * sizeof(double));
    double* Vw = (double*)malloc((size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1) * sizeof(double));
    double* sv = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int64_t* perm = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!W || !Vw || !sv || !perm) {
        free(W);
        free(Vw);
        free(sv);
        free(perm);
        return ORC_ENOMEM;
    }
    for (int64_t j = 0; j < n; ++j) memcpy(W + IDX(0, j, m), A + IDX(0, j, lda), (size_t)m * sizeof(double));
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) Vw[IDX(i, j, n)] = i == j ? 1.0 : 0.0;

    const double tol = (double)m * ldexp(1.0, -53);
    int sweep = 0, converged = (n < 2);
    while (!converged && sweep < max_sweeps) {
        int rotated = 0;
        for (int64_t p = 0; p + 1 < n; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                double* wp = W + IDX(0, p, m);
                double* wq = W + IDX(0, q, m);
                double alpha = dot(wp, wp, m);
                double beta = dot(wq, wq, m);
                double gamma = dot(wp, wq, m);
                if (alpha == 0.0 || beta == 0.0) continue;
                if (fabs(gamma) <= tol * sqrt(alpha) * sqrt(beta)) continue;
                rotated = 1;
                double zeta = (beta - alpha) / (2.0 * gamma);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double sn = c * t;
                for (int64_t i = 0; i < m; ++i) {
                    double a = wp[i], b = wq[i];
                    wp[i] = c * a - sn * b;
                    wq[i] = sn * a + c * b;
                }
                double* vp = Vw + IDX(0, p, n);
                double* vq = Vw + IDX(0, q, n);
                for (int64_t i = 0; i < n; ++i) {
                    double a = vp[i], b = vq[i];
                    vp[i] = c * a - sn * b;
                    vq[i] = sn * a + c * b;
                }
            }
        }
        ++sweep;
        if (!rotated) converged = 1;
    }
    if (sweeps_out) *sweeps_out = sweep;

    for (int64_t j = 0; j < n; ++j) {
        sv[j] = sqrt(dot(W + IDX(0, j, m), W + IDX(0, j, m), m));
        perm[j] = j;
    }
    /* Stable insertion sort, descending. */
    for (int64_t a = 1; a < n; ++a) {
        int64_t pj = perm[a];
        int64_t b = a - 1;
        while (b >= 0 && sv[perm[b]] < sv[pj]) {
            perm[b + 1] = perm[b];
            --b;
        }
        perm[b + 1] = pj;
    }
    for (int64_t j = 0; j < n; ++j) {
        int64_t src = perm[j];
        double sj = sv[src];
        s[j] = sj;
        if (U) {
            double* u = U + IDX(0, j, m);
            const double* w = W + IDX(0, src, m);
            for (int64_t i = 0; i < m; ++i) u[i] = sj > 0.0 ? w[i] / sj : 0.0;
        }
        if (V) memcpy(V + IDX(0, j, n), Vw + IDX(0, src, n), (size_t)n * sizeof(double));
    }
    free(W);
    free(Vw);
    free(sv);
    free(perm);
    return converged ? ORC_OK : ORC_ENOCONV;
}

/*
 * Sign convention for a small factor: each of the first k columns of X
 * (rows x cols, ld rows) gets its largest-magnitude entry (lowest index on
 * ties) non-negative.  The flip is recorded in flip[j] (+1 / -1).
 */
static void sign_rule(int64_t rows, int64_t k, double* X, int64_t ldx, double* flip)
{
    for (int64_t j = 0; j < k; ++j) {
        double* x = X + IDX(0, j, ldx);
        int64_t best = 0;
        double bv = -1.0;
        for (int64_t i = 0; i < rows; ++i)
            if (fabs(x[i]) > bv) {
                bv = fabs(x[i]);
                best = i;
            }
        double f = (rows > 0 && x[best] < 0.0) ? -1.0 : 1.0;
        if (f < 0.0)
            for (int64_t i = 0; i < rows; ++i) x[i] = -x[i];
        if (flip) flip[j] = f;
    }
}

/* ------------------------------------------------------------------------ */
/* One batch of Algorithm 1.                                                */
/* ------------------------------------------------------------------------ */

/* Build the panel C = [ff * U * diag(s) | A] (M x n, ld M). */
static double* build_panel(int64_t M, int64_t r, double ff, const double* U, int64_t ldu, const double* s,
                           const double* A, int64_t N, int64_t lda)
{
    int64_t n = r + N;
    double* C = (double*)malloc((size_t)M * (size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!C) return NULL;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        double* c = C + IDX(0, j, M);
        if (j < r) {
            double a = ff * s[j];
            const double* u = U + IDX(0, j, ldu);
            for (int64_t i = 0; i < M; ++i) c[i] = a * u[i];
        } else {
            memcpy(c, A + IDX(0, j - r, lda), (size_t)M * sizeof(double));
        }
    }
    return C;
}

/*
 * Deterministic step: Q R = C (Householder), R = Ut S Vt^T (Jacobi),
 * keep r' = min(K, n) leading triplets, U <- Q Ut[:, :r'] after the sign
 * rule on Ut.  (Algorithm 1: the per-batch update; the initialisation when r = 0.)
 */
static int step_det(int64_t M, int32_t K, const double* C, int64_t n, double* U, int64_t ldu, double* s,
                    int32_t* r_out, double* smallU_out)
{
    double* Q = (double*)malloc((size_t)M * (size_t)n * sizeof(double));
    double* R = (double*)malloc((size_t)n * (size_t)n * sizeof(double));
    double* Ut = (double*)malloc((size_t)n * (size_t)n * sizeof(double));
    double* S = (double*)malloc((size_t)n * sizeof(double));
    int rc = ORC_ENOMEM;
    if (!Q || !R || !Ut || !S) goto done;
    rc = orc_hhqr(M, n, C, M, Q, R);
    if (rc) goto done;
    rc = orc_jacobi_svd(n, n, R, n, Ut, S, NULL, 60, NULL);
    if (rc) goto done;
    {
        int64_t rk = K < n ? K : n;
        sign_rule(n, rk, Ut, n, NULL);
        mm_nn(M, rk, n, Q, M, Ut, n, U, ldu);
        for (int64_t j = 0; j < rk; ++j) s[j] = S[j];
        *r_out = (int32_t)rk;
        if (smallU_out) memcpy(smallU_out, Ut, (size_t)n * (size_t)rk * sizeof(double));
    }
done:
    free(Q);
    free(R);
    free(Ut);
    free(S);
    return rc;
}

/*
 * Randomized step with test matrix Omega (n x ell), ell < n:
 *   Y = C Omega, Q = qr(Y);
 *   q times: Z = C^T Q, Qz = qr(Z), Y = C Qz, Q = qr(Y);
 *   B = Q^T C (ell x n);  B = Ut S Vt^T (Jacobi on B^T);
 *   U <- Q Ut[:, :K], s <- S[:K]  (Eqs. (7)-(11)).
 */
static int step_rand(int64_t M, int32_t K, int32_t q, const double* C, int64_t n, const double* Om, int64_t ell,
                     double* U, int64_t ldu, double* s, int32_t* r_out, double* smallU_out)
{
    double* Y = (double*)malloc((size_t)M * (size_t)ell * sizeof(double));
    double* Q = (double*)malloc((size_t)M * (size_t)ell * sizeof(double));
    double* Ry = (double*)malloc((size_t)ell * (size_t)ell * sizeof(double));
    double* Z = (double*)malloc((size_t)n * (size_t)ell * sizeof(double));
    double* Qz = (double*)malloc((size_t)n * (size_t)ell * sizeof(double));
    double* Bt = (double*)malloc((size_t)n * (size_t)ell * sizeof(double));
    double* S = (double*)malloc((size_t)ell * sizeof(double));
    double* Vb = (double*)malloc((size_t)ell * (size_t)ell * sizeof(double));
    int rc = ORC_ENOMEM;
    if (!Y || !Q || !Ry || !Z || !Qz || !Bt || !S || !Vb) goto done;
    mm_nn(M, ell, n, C, M, Om, n, Y, M);
    rc = orc_hhqr(M, ell, Y, M, Q, Ry);
    if (rc) goto done;
    for (int32_t it = 0; it < q; ++it) {
        rc = mm_tn(n, ell, M, C, M, Q, M, Z, n);
        if (rc) goto done;
        rc = orc_hhqr(n, ell, Z, n, Qz, Ry);
        if (rc) goto done;
        mm_nn(M, ell, n, C, M, Qz, n, Y, M);
        rc = orc_hhqr(M, ell, Y, M, Q, Ry);
        if (rc) goto done;
    }
    /* B^T = C^T Q (n x ell). */
    rc = mm_tn(n, ell, M, C, M, Q, M, Bt, n);
    if (rc) goto done;
    /* B^T = W S Vb^T  =>  B = Vb S W^T: the left factor of B is Vb. */
    rc = orc_jacobi_svd(n, ell, Bt, n, NULL, S, Vb, 60, NULL);
    if (rc) goto done;
    {
        int64_t rk = K < ell ? K : ell;
        sign_rule(ell, rk, Vb, ell, NULL);
        mm_nn(M, rk, ell, Q, M, Vb, ell, U, ldu);
        for (int64_t j = 0; j < rk; ++j) s[j] = S[j];
        *r_out = (int32_t)rk;
        if (smallU_out) memcpy(smallU_out, Vb, (size_t)ell * (size_t)rk * sizeof(double));
    }
done:
    free(Y);
    free(Q);
    free(Ry);
    free(Z);
    free(Qz);
    free(Bt);
    free(S);
    free(Vb);
    return rc;
}

/*
 * One batch of the streaming SVD.  State: U (M x K capacity, ld ldu), s (K),
 * *r current rank (0 before the first batch).  A: M x N (ld lda).  With
 * Omega == NULL or ell >= r + N the deterministic step runs; otherwise the
 * randomized step with the given (r + N) x ell test matrix.
 * Requires M >= r + N.  smallU_out (optional) receives the retained columns
 * of the small left factor after the sign rule.
 */
int orc_stream_update(int64_t M, int32_t K, double ff, int32_t ell, int32_t q, double* U, int64_t ldu, double* s,
                      int32_t* r, const double* A, int64_t N, int64_t lda, const double* Omega, double* smallU_out)
{
    if (M < 1 || K < 1 || N < 0 || !(ff > 0.0 && ff <= 1.0) || q < 0) return ORC_EINVAL;
    int64_t r0 = *r;
    int64_t n = r0 + N;
    if (N == 0) return ORC_OK;
    if (M < n) return ORC_EINVAL;
    double* C = build_panel(M, r0, ff, U, ldu, s, A, N, lda);
    if (!C) return ORC_ENOMEM;
    int rc;
    if (Omega == NULL || ell <= 0 || ell >= n) rc = step_det(M, K, C, n, U, ldu, s, r, smallU_out);
    else rc = step_rand(M, K, q, C, n, Omega, ell, U, ldu, s, r, smallU_out);
    free(C);
    return rc;
}

/*
 * Low-rank SVD of a small m x n matrix A (ld lda), Eqs. (7)-(11) without power
 * iterations, with the Gaussian test matrix Om (n x ell, 1 <= ell <= min(m, n)):
 * Y = A Om, Q = qr(Y), B = Q^T A, B = Ut S Vt^T (Jacobi on B^T), U = Q Ut[:, :k]
 * and s = S[:k] with k = min(K, ell), the sign rule on Ut.  (The randomized step
 * of the stream with q = 0.)  Exact when rank(A) <= ell.
 */
int orc_low_rank_svd(int64_t m, int64_t n, const double* A, int64_t lda, int32_t K, const double* Om, int64_t ell,
                     double* U, int64_t ldu, double* s, int32_t* k_out)
{
    if (m < 1 || n < 1 || K < 1 || ell < 1 || ell > m || ell > n || lda < m) return ORC_EINVAL;
    double* C = (double*)malloc((size_t)m * (size_t)n * sizeof(double));
    if (!C) return ORC_ENOMEM;
    for (int64_t j = 0; j < n; ++j) memcpy(C + IDX(0, j, m), A + IDX(0, j, lda), (size_t)m * sizeof(double));
    int rc = step_rand(m, K, 0, C, n, Om, ell, U, ldu, s, k_out, NULL);
    free(C);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* APMOS: Algorithm 2, Eqs. (3)-(6).                                        */
/* ------------------------------------------------------------------------ */

/*
 * P partitions A^i (M_i x N, ld M_i, stacked one after another in A_all).
 *   1. local SVD: Q_i R_i = A^i (Householder), R_i = . S_i V_i^T (Jacobi);
 *   2. W_i = V_i[:, :rloc] diag(S_i[:rloc]);  W = [W_1 ... W_P]  (N x P*rloc);
 *   3. W = X Lambda Y^T;  X~ = X[:, :K] (sign rule), Lambda~ = Lambda[:K];
 *   4. U^i = A^i X~ diag(1 / Lambda~)   (written stacked into U_all, ld M_i).
 * Returns ORC_EINVAL if Lambda~_K <= N * 2^-53 * Lambda~_1.
 */
static int apmos_impl(int32_t P, const int64_t* M_parts, int64_t N, int32_t rloc, int32_t K, const double* A_all,
                      const double* Om, int64_t ell, double* U_all, double* Lambda, double* X_out)
{
    if (P < 1 || N < 1 || rloc < 1 || rloc > N || K < 1 || K > N) return ORC_EINVAL;
    int64_t wcols = (int64_t)P * rloc;
    if (K > wcols) return ORC_EINVAL;
    if (Om && (ell < K || ell > N || ell > wcols)) return ORC_EINVAL;
    double* Wm = (double*)calloc((size_t)N * (size_t)wcols, sizeof(double));
    if (!Wm) return ORC_ENOMEM;
    int rc = ORC_OK;
    int64_t off = 0;
    for (int32_t i = 0; i < P && rc == ORC_OK; ++i) {
        int64_t Mi = M_parts[i];
        if (Mi < N) {
            rc = ORC_EINVAL;
            break;
        }
        double* Q = (double*)malloc((size_t)Mi * (size_t)N * sizeof(double));
        double* R = (double*)malloc((size_t)N * (size_t)N * sizeof(double));
        double* S = (double*)malloc((size_t)N * sizeof(double));
        double* V = (double*)malloc((size_t)N * (size_t)N * sizeof(double));
        if (!Q || !R || !S || !V) rc = ORC_ENOMEM;
        if (rc == ORC_OK) rc = orc_hhqr(Mi, N, A_all + off, Mi, Q, R);
        if (rc == ORC_OK) rc = orc_jacobi_svd(N, N, R, N, NULL, S, V, 60, NULL);
        /* the sign rule on the kept right vectors: W's column signs do not change
         * W W^T (the exact SVD of W), but they do change the low-rank SVD's sketch W Om */
        if (rc == ORC_OK) sign_rule(N, rloc, V, N, NULL);
        if (rc == ORC_OK)
            for (int32_t j = 0; j < rloc; ++j)
                for (int64_t k = 0; k < N; ++k) Wm[IDX(k, (int64_t)i * rloc + j, N)] = V[IDX(k, j, N)] * S[j];
        free(Q);
        free(R);
        free(S);
        free(V);
        off += Mi * N;
    }
    double* Xf = NULL;
    double* Lf = NULL;
    if (rc == ORC_OK) {
        Xf = (double*)malloc((size_t)N * (size_t)N * sizeof(double));
        int64_t nl = wcols < N ? wcols : N;
        Lf = (double*)malloc((size_t)N * sizeof(double));
        if (!Xf || !Lf) rc = ORC_ENOMEM;
        if (rc == ORC_OK && Om) {
            /* the low-rank SVD of W (sign rule on its small factor) */
            int32_t kk = 0;
            rc = orc_low_rank_svd(N, wcols, Wm, N, K, Om, ell, Xf, N, Lf, &kk);
        } else if (rc == ORC_OK) {
            if (wcols >= N) {
                /* W^T (wcols x N) = Uw S Vw^T  =>  W = Vw S Uw^T: X = Vw. */
                double* Wt = (double*)malloc((size_t)wcols * (size_t)N * sizeof(double));
                if (!Wt) rc = ORC_ENOMEM;
                else {
                    for (int64_t a = 0; a < N; ++a)
                        for (int64_t b = 0; b < wcols; ++b) Wt[IDX(b, a, wcols)] = Wm[IDX(a, b, N)];
                    rc = orc_jacobi_svd(wcols, N, Wt, wcols, NULL, Lf, Xf, 60, NULL);
                    free(Wt);
                }
            } else {
                /* W (N x wcols) tall: W = X S Vw^T directly. */
                rc = orc_jacobi_svd(N, wcols, Wm, N, Xf, Lf, NULL, 60, NULL);
            }
        }
        (void)nl;
    }
    if (rc == ORC_OK) {
        if (!(Lf[K - 1] > (double)N * ldexp(1.0, -53) * Lf[0])) rc = ORC_EINVAL;
    }
    if (rc == ORC_OK) {
        if (!Om) sign_rule(N, K, Xf, N, NULL);
        double* T = (double*)malloc((size_t)N * (size_t)K * sizeof(double));
        if (!T) rc = ORC_ENOMEM;
        else {
            for (int32_t j = 0; j < K; ++j)
                for (int64_t k = 0; k < N; ++k) T[IDX(k, j, N)] = Xf[IDX(k, j, N)] / Lf[j];
            off = 0;
            int64_t uoff = 0;
            for (int32_t i = 0; i < P; ++i) {
                int64_t Mi = M_parts[i];
                mm_nn(Mi, K, N, A_all + off, Mi, T, N, U_all + uoff, Mi);
                off += Mi * N;
                uoff += Mi * K;
            }
            free(T);
            for (int32_t j = 0; j < K; ++j) Lambda[j] = Lf[j];
            if (X_out) memcpy(X_out, Xf, (size_t)N * (size_t)K * sizeof(double));
        }
    }
    free(Xf);
    free(Lf);
    free(Wm);
    return rc;
}

int orc_apmos(int32_t P, const int64_t* M_parts, int64_t N, int32_t rloc, int32_t K, const double* A_all,
              double* U_all, double* Lambda, double* X_out)
{
    return apmos_impl(P, M_parts, N, rloc, K, A_all, NULL, 0, U_all, Lambda, X_out);
}

/*
 * Algorithm 2 with the global SVD of W (step 4) taken by the low-rank SVD of
 * Eqs. (7)-(11) with the test matrix Om (P*rloc x ell, K <= ell <= N), as the
 * paper's parallel listing does when randomization is on.
 */
int orc_apmos_lr(int32_t P, const int64_t* M_parts, int64_t N, int32_t rloc, int32_t K, const double* A_all,
                 const double* Om, int64_t ell, double* U_all, double* Lambda, double* X_out)
{
    if (!Om) return ORC_EINVAL;
    return apmos_impl(P, M_parts, N, rloc, K, A_all, Om, ell, U_all, Lambda, X_out);
}

/* ------------------------------------------------------------------------ */
/* Partitioned streaming: the parallel update of Section 3 (row partitions). */
/* ------------------------------------------------------------------------ */

/*
 * One batch of the partitioned streaming SVD over P row partitions.  State:
 * U_all holds U^i (M_i x K capacity, ld M_i) stacked one after another, s (K),
 * *r the current rank.  A_all holds the batch partitions A^i (M_i x N, ld M_i)
 * stacked the same way.  Per batch:
 *   1. local panels C^i = [ff U^i diag(s) | A^i] and local Householder QR
 *      C^i = Q^i R^i (R^i: n x n; requires M_i >= n);
 *   2. the R^i stacked (P n x n) and factored again, [R^1; ..; R^P] = Q_g R_f;
 *   3. R_f = U~ S V~^T (Jacobi), descending; keep r' = min(K, n) triplets,
 *      sign rule on U~;
 *   4. U^i <- Q^i Q_g^i U~[:, :r'], with Q_g^i the i-th n-row block of Q_g.
 * In exact arithmetic this is the serial update of the stacked panel: R_f
 * is the R factor of the whole panel (both with a non-negative diagonal).
 */
static int pstream_impl(int32_t P, const int64_t* M_parts, int32_t K, double ff, double* U_all, double* s,
                        int32_t* r, const double* A_all, int64_t N, const double* Om, int64_t ell)
{
    if (P < 1 || K < 1 || N < 0 || !(ff > 0.0 && ff <= 1.0)) return ORC_EINVAL;
    const int64_t r0 = *r, n = r0 + N;
    if (N == 0) return ORC_OK;
    if (Om && (ell < 1 || ell > n)) return ORC_EINVAL;
    for (int32_t i = 0; i < P; ++i)
        if (M_parts[i] < n) return ORC_EINVAL;
    const int64_t pn = (int64_t)P * n;
    double* Rs = (double*)calloc((size_t)pn * (size_t)n, sizeof(double));
    double** Qs = (double**)calloc((size_t)P, sizeof(double*));
    double* Qg = (double*)malloc((size_t)pn * (size_t)n * sizeof(double));
    double* Rf = (double*)malloc((size_t)n * (size_t)n * sizeof(double));
    double* Ut = (double*)malloc((size_t)n * (size_t)n * sizeof(double));
    double* S = (double*)malloc((size_t)n * sizeof(double));
    int rc = (Rs && Qs && Qg && Rf && Ut && S) ? ORC_OK : ORC_ENOMEM;
    /* 1. local panels and local QR */
    int64_t off = 0, uoff = 0;
    for (int32_t i = 0; i < P && rc == ORC_OK; ++i) {
        const int64_t Mi = M_parts[i];
        double* C = build_panel(Mi, r0, ff, U_all + uoff, Mi, s, A_all + off, N, Mi);
        double* R = (double*)malloc((size_t)n * (size_t)n * sizeof(double));
        Qs[i] = (double*)malloc((size_t)Mi * (size_t)n * sizeof(double));
        if (!C || !R || !Qs[i]) rc = ORC_ENOMEM;
        if (rc == ORC_OK) rc = orc_hhqr(Mi, n, C, Mi, Qs[i], R);
        if (rc == ORC_OK)
            for (int64_t j = 0; j < n; ++j)
                for (int64_t a = 0; a < n; ++a) Rs[IDX((int64_t)i * n + a, j, pn)] = R[IDX(a, j, n)];
        free(C);
        free(R);
        off += Mi * N;
        uoff += Mi * K;
    }
    /* 2. QR of the stacked R factors */
    if (rc == ORC_OK) rc = orc_hhqr(pn, n, Rs, pn, Qg, Rf);
    /* 3. SVD of the combined R: exact (Jacobi), or the low-rank SVD of
     * Eqs. (7)-(11) with the test matrix Om (n x ell; sign rule on its small factor) */
    int64_t rk = K < n ? K : n;
    if (rc == ORC_OK && Om) {
        int32_t kk = 0;
        rc = orc_low_rank_svd(n, n, Rf, n, K, Om, ell, Ut, n, S, &kk);
        rk = kk;
    } else if (rc == ORC_OK) {
        rc = orc_jacobi_svd(n, n, Rf, n, Ut, S, NULL, 60, NULL);
        if (rc == ORC_OK) sign_rule(n, rk, Ut, n, NULL);
    }
    if (rc == ORC_OK) {
        /* 4. U^i = Q^i (Q_g^i U~_rk) */
        double* T = (double*)malloc((size_t)n * (size_t)rk * sizeof(double));
        double* Qgi = (double*)malloc((size_t)n * (size_t)n * sizeof(double));
        if (!T || !Qgi) rc = ORC_ENOMEM;
        uoff = 0;
        for (int32_t i = 0; i < P && rc == ORC_OK; ++i) {
            const int64_t Mi = M_parts[i];
            for (int64_t j = 0; j < n; ++j)
                for (int64_t a = 0; a < n; ++a) Qgi[IDX(a, j, n)] = Qg[IDX((int64_t)i * n + a, j, pn)];
            mm_nn(n, rk, n, Qgi, n, Ut, n, T, n);
            mm_nn(Mi, rk, n, Qs[i], Mi, T, n, U_all + uoff, Mi);
            uoff += Mi * K;
        }
        free(T);
        free(Qgi);
        if (rc == ORC_OK) {
            for (int64_t j = 0; j < rk; ++j) s[j] = S[j];
            *r = (int32_t)rk;
        }
    }
    if (Qs)
        for (int32_t i = 0; i < P; ++i) free(Qs[i]);
    free(Qs);
    free(Rs);
    free(Qg);
    free(Rf);
    free(Ut);
    free(S);
    return rc;
}

int orc_pstream_update(int32_t P, const int64_t* M_parts, int32_t K, double ff, double* U_all, double* s, int32_t* r,
                       const double* A_all, int64_t N)
{
    return pstream_impl(P, M_parts, K, ff, U_all, s, r, A_all, N, NULL, 0);
}

/*
 * The partitioned update with the SVD of the combined R factor (step 3) taken
 * by the low-rank SVD of Eqs. (7)-(11) with the test matrix Om (n x ell),
 * n = r + N, as the paper's parallel QR listing does when randomization is on.
 * The rank kept is min(K, ell).
 */
int orc_pstream_update_lr(int32_t P, const int64_t* M_parts, int32_t K, double ff, double* U_all, double* s,
                          int32_t* r, const double* A_all, int64_t N, const double* Om, int64_t ell)
{
    if (!Om) return ORC_EINVAL;
    return pstream_impl(P, M_parts, K, ff, U_all, s, r, A_all, N, Om, ell);
}

/* ------------------------------------------------------------------------ */
/* Loss and its reverse-mode gradient through the deterministic stream.     */
/* ------------------------------------------------------------------------ */

/*
 * Forward pass of the deterministic stream over B batches of Nb columns
 * each (A: M x B*Nb, ld lda), storing the state entering every batch in
 * Ust (B x M x K) / sst (B x K) / rst (B) when they are not NULL.  Final
 * state in U (M x K, ld M), s, *r.
 */
static int stream_forward(int64_t M, int32_t K, double ff, int32_t B, int64_t Nb, const double* A, int64_t lda,
                          double* U, double* s, int32_t* r, double* Ust, double* sst, int32_t* rst)
{
    *r = 0;
    for (int32_t b = 0; b < B; ++b) {
        if (Ust) {
            memcpy(Ust + (size_t)b * (size_t)M * (size_t)K, U, (size_t)M * (size_t)K * sizeof(double));
            memcpy(sst + (size_t)b * (size_t)K, s, (size_t)K * sizeof(double));
            rst[b] = *r;
        }
        int rc = orc_stream_update(M, K, ff, 0, 0, U, M, s, r, A + IDX(0, (int64_t)b * Nb, lda), Nb, lda, NULL, NULL);
        if (rc) return rc;
    }
    return ORC_OK;
}

/*
 * Loss of the streamed truncated SVD:
 *   L = ||A - U U^T A||_F^2 + sum_{j<r} w_j s_j,
 * evaluated as ||A||^2 - ||U^T A||^2 + sum w_j s_j (U has orthonormal
 * columns).  Also returns the final U, s (optional).
 */
int orc_stream_loss(int64_t M, int32_t K, double ff, int32_t B, int64_t Nb, const double* A, int64_t lda,
                    const double* w, double* loss, double* U_out, double* s_out)
{
    double* U = (double*)calloc((size_t)M * (size_t)K, sizeof(double));
    double* s = (double*)calloc((size_t)K, sizeof(double));
    int64_t Nt = (int64_t)B * Nb;
    double* UtA = (double*)malloc((size_t)K * (size_t)(Nt > 0 ? Nt : 1) * sizeof(double));
    int32_t r = 0;
    int rc = ORC_ENOMEM;
    if (!U || !s || !UtA) goto done;
    rc = stream_forward(M, K, ff, B, Nb, A, lda, U, s, &r, NULL, NULL, NULL);
    if (rc) goto done;
    rc = mm_tn(r, Nt, M, U, M, A, lda, UtA, K);
    if (rc) goto done;
    {
        double a2 = 0.0, p2 = 0.0, ws = 0.0;
        for (int64_t j = 0; j < Nt; ++j) a2 += dot(A + IDX(0, j, lda), A + IDX(0, j, lda), M);
        for (int64_t j = 0; j < Nt; ++j)
            for (int32_t i = 0; i < r; ++i) p2 += UtA[IDX(i, j, K)] * UtA[IDX(i, j, K)];
        for (int32_t i = 0; i < r; ++i) ws += w[i] * s[i];
        *loss = a2 - p2 + ws;
    }
    if (U_out) memcpy(U_out, U, (size_t)M * (size_t)K * sizeof(double));
    if (s_out) memcpy(s_out, s, (size_t)K * sizeof(double));
done:
    free(U);
    free(s);
    free(UtA);
    return rc;
}

/*
 * Adjoint of one truncated-SVD step.  C (M x n) = Uf S V^T is the full thin
 * SVD (Uf = Q Ut, V = Vt from the QR of C and the Jacobi SVD of R, with the
 * sign rule applied to the first rk columns of Ut and V alike).  Given the
 * cotangents Ub (M x rk) of the retained columns of Uf and sb (rk) of the
 * retained singular values, returns
 *   Cb = Uf [diag(sb) + (F o (Uf^T Ub - Ub^T Uf)) S] V^T
 *        + (I - Uf Uf^T) Ub S^-1 V^T,     F_ij = 1 / (s_j^2 - s_i^2),
 * where Ub and sb are padded with zeros beyond rk (pairs with both indices
 * >= rk carry no cotangent and are skipped).
 */
static int svd_step_adjoint(int64_t M, int32_t K, const double* C, int64_t n, const double* Ub, const double* sb,
                            double* Cb)
{
    int64_t rk = K < n ? K : n;
    double* Q = (double*)malloc((size_t)M * (size_t)n * sizeof(double));
    double* R = (double*)malloc((size_t)n * (size_t)n * sizeof(double));
    double* Ut = (double*)malloc((size_t)n * (size_t)n * sizeof(double));
    double* Vt = (double*)malloc((size_t)n * (size_t)n * sizeof(double));
    double* S = (double*)malloc((size_t)n * sizeof(double));
    double* flip = (double*)malloc((size_t)n * sizeof(double));
    double* Uf = (double*)malloc((size_t)M * (size_t)n * sizeof(double));
    double* G = (double*)malloc((size_t)n * (size_t)rk * sizeof(double));   /* Uf^T Ub */
    double* In = (double*)calloc((size_t)n * (size_t)n, sizeof(double));    /* inner n x n */
    double* T1 = (double*)malloc((size_t)n * (size_t)n * sizeof(double));   /* inner V^T */
    double* Pn = (double*)malloc((size_t)M * (size_t)rk * sizeof(double));  /* (I-UU^T) Ub S^-1 */
    double* T2 = (double*)malloc((size_t)rk * (size_t)n * sizeof(double));
    int rc = ORC_ENOMEM;
    if (!Q || !R || !Ut || !Vt || !S || !flip || !Uf || !G || !In || !T1 || !Pn || !T2) goto done;
    rc = orc_hhqr(M, n, C, M, Q, R);
    if (rc) goto done;
    rc = orc_jacobi_svd(n, n, R, n, Ut, S, Vt, 60, NULL);
    if (rc) goto done;
    sign_rule(n, rk, Ut, n, flip);
    for (int64_t j = 0; j < rk; ++j)
        if (flip[j] < 0.0)
            for (int64_t i = 0; i < n; ++i) Vt[IDX(i, j, n)] = -Vt[IDX(i, j, n)];
    mm_nn(M, n, n, Q, M, Ut, n, Uf, M);
    rc = mm_tn(n, rk, M, Uf, M, Ub, M, G, n);
    if (rc) goto done;
    /* Inner = diag(sb) + (F o (G - G^T)) S ; G padded: G_ij = 0 for j >= rk. */
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < n; ++i) {
            if (i == j) {
                In[IDX(i, j, n)] = j < rk ? sb[j] : 0.0;
                continue;
            }
            if (i >= rk && j >= rk) continue;
            double gij = j < rk ? G[IDX(i, j, n)] : 0.0;
            double gji = i < rk ? G[IDX(j, i, n)] : 0.0;
            double f = 1.0 / (S[j] * S[j] - S[i] * S[i]);
            In[IDX(i, j, n)] = f * (gij - gji) * S[j];
        }
    }
    /* T1 = In V^T ; Cb = Uf T1. */
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k) acc += In[IDX(i, k, n)] * Vt[IDX(j, k, n)];
            T1[IDX(i, j, n)] = acc;
        }
    mm_nn(M, n, n, Uf, M, T1, n, Cb, M);
    /* Pn = (Ub - Uf G) S^-1 (first rk columns). */
    mm_nn(M, rk, n, Uf, M, G, n, Pn, M);
    for (int64_t j = 0; j < rk; ++j) {
        double inv = 1.0 / S[j];
        double* p = Pn + IDX(0, j, M);
        const double* ub = Ub + IDX(0, j, M);
        for (int64_t i = 0; i < M; ++i) p[i] = (ub[i] - p[i]) * inv;
    }
    /* Cb += Pn V[:, :rk]^T. */
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < rk; ++i) T2[IDX(i, j, rk)] = Vt[IDX(j, i, n)];
    {
        double* tmp = (double*)malloc((size_t)M * (size_t)n * sizeof(double));
        if (!tmp) {
            rc = ORC_ENOMEM;
            goto done;
        }
        mm_nn(M, n, rk, Pn, M, T2, rk, tmp, M);
        for (size_t e = 0; e < (size_t)M * (size_t)n; ++e) Cb[e] += tmp[e];
        free(tmp);
    }
    rc = ORC_OK;
done:
    free(Q);
    free(R);
    free(Ut);
    free(Vt);
    free(S);
    free(flip);
    free(Uf);
    free(G);
    free(In);
    free(T1);
    free(Pn);
    free(T2);
    return rc;
}

/*
 * Gradient dL/dA (M x B*Nb, ld M) of orc_stream_loss.  Direct term
 * 2 (I - U U^T) A; the final state receives the cotangents
 * Ub = -2 A A^T U and sb = w, which are carried back through every batch
 * (recomputing that batch's panel from the stored incoming state) with
 * svd_step_adjoint; the panel cotangent splits into the data part (added to
 * the gradient of that batch) and the part of ff*U*diag(s), giving
 * Ub_prev = ff * Cb_U diag(s_prev) and sb_prev_j = ff * u_prev_j^T cb_j.
 */
int orc_stream_grad(int64_t M, int32_t K, double ff, int32_t B, int64_t Nb, const double* A, int64_t lda,
                    const double* w, double* grad)
{
    int64_t Nt = (int64_t)B * Nb;
    double* U = (double*)calloc((size_t)M * (size_t)K, sizeof(double));
    double* s = (double*)calloc((size_t)K, sizeof(double));
    double* Ust = (double*)calloc((size_t)B * (size_t)M * (size_t)K, sizeof(double));
    double* sst = (double*)calloc((size_t)B * (size_t)K, sizeof(double));
    int32_t* rst = (int32_t*)calloc((size_t)B, sizeof(int32_t));
    double* UtA = (double*)malloc((size_t)K * (size_t)Nt * sizeof(double));
    double* Ub = (double*)calloc((size_t)M * (size_t)K, sizeof(double));
    double* sb = (double*)calloc((size_t)K, sizeof(double));
    int32_t r = 0;
    int rc = ORC_ENOMEM;
    if (!U || !s || !Ust || !sst || !rst || !UtA || !Ub || !sb) goto done;
    rc = stream_forward(M, K, ff, B, Nb, A, lda, U, s, &r, Ust, sst, rst);
    if (rc) goto done;
    rc = mm_tn(r, Nt, M, U, M, A, lda, UtA, K);
    if (rc) goto done;
    /* Direct term: grad = 2 A - 2 U (U^T A). */
    {
        double* UUA = (double*)malloc((size_t)M * (size_t)Nt * sizeof(double));
        if (!UUA) {
            rc = ORC_ENOMEM;
            goto done;
        }
        mm_nn(M, Nt, r, U, M, UtA, K, UUA, M);
        for (int64_t j = 0; j < Nt; ++j)
            for (int64_t i = 0; i < M; ++i) grad[IDX(i, j, M)] = 2.0 * A[IDX(i, j, lda)] - 2.0 * UUA[IDX(i, j, M)];
        free(UUA);
    }
    /* Ub = -2 A (A^T U) ; sb = w. */
    {
        double* AtU = (double*)malloc((size_t)Nt * (size_t)K * sizeof(double));
        if (!AtU) {
            rc = ORC_ENOMEM;
            goto done;
        }
        for (int32_t j = 0; j < r; ++j)
            for (int64_t i = 0; i < Nt; ++i) AtU[IDX(i, j, Nt)] = UtA[IDX(j, i, K)];
        mm_nn(M, r, Nt, A, lda, AtU, Nt, Ub, M);
        for (size_t e = 0; e < (size_t)M * (size_t)r; ++e) Ub[e] *= -2.0;
        for (int32_t j = 0; j < r; ++j) sb[j] = w[j];
        free(AtU);
    }
    for (int32_t b = B - 1; b >= 0; --b) {
        const double* Up = Ust + (size_t)b * (size_t)M * (size_t)K;
        const double* sp = sst + (size_t)b * (size_t)K;
        int64_t rp = rst[b];
        int64_t n = rp + Nb;
        double* C = build_panel(M, rp, ff, Up, M, sp, A + IDX(0, (int64_t)b * Nb, lda), Nb, lda);
        double* Cb = (double*)malloc((size_t)M * (size_t)n * sizeof(double));
        if (!C || !Cb) {
            free(C);
            free(Cb);
            rc = ORC_ENOMEM;
            goto done;
        }
        rc = svd_step_adjoint(M, K, C, n, Ub, sb, Cb);
        if (rc) {
            free(C);
            free(Cb);
            goto done;
        }
        for (int64_t j = 0; j < Nb; ++j)
            for (int64_t i = 0; i < M; ++i) grad[IDX(i, (int64_t)b * Nb + j, M)] += Cb[IDX(i, rp + j, M)];
        memset(Ub, 0, (size_t)M * (size_t)K * sizeof(double));
        memset(sb, 0, (size_t)K * sizeof(double));
        for (int64_t j = 0; j < rp; ++j) {
            const double* cb = Cb + IDX(0, j, M);
            const double* u = Up + IDX(0, j, M);
            double* ub = Ub + IDX(0, j, M);
            for (int64_t i = 0; i < M; ++i) ub[i] = ff * sp[j] * cb[i];
            sb[j] = ff * dot(u, cb, M);
        }
        free(C);
        free(Cb);
    }
    rc = ORC_OK;
done:
    free(U);
    free(s);
    free(Ust);
    free(sst);
    free(rst);
    free(UtA);
    free(Ub);
    free(sb);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Utilities exported for the tests.                                        */
/* ------------------------------------------------------------------------ */

void orc_matmul_nn(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, const double* B, int64_t ldb,
                   double* C, int64_t ldc)
{
    mm_nn(m, n, k, A, lda, B, ldb, C, ldc);
}

int orc_matmul_tn(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, const double* B, int64_t ldb,
                  double* C, int64_t ldc)
{
    return mm_tn(m, n, k, A, lda, B, ldb, C, ldc);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
