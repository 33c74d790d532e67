// psvd_host.hip -- C ABI, handle state and the per-batch orchestration.
//
// One update (Algorithm 1 of Sec. 3.1) is a fixed sequence of kernels on the
// handle's stream; no step waits for the host.  The panel C = [ff U diag(s) | A]
// is never formed: kernels read [U | A] and the column scale D = ff diag(s) is
// applied to the small operands (G = D G' D, X' = D X, P = D P', T' = D T).
//
// Deterministic step (QR of C + SVD of R):
//   G' = [U|A]^T [U|A]  ->  R1 = chol(D G' D)       (eigen route on breakdown)
//   G2 = (C R1^-1)^T (C R1^-1) -> R2 = chol(G2), R = R2 R1   (Cholesky-QR2)
//   R = U~ S V~^T (one-sided Jacobi), keep K, sign rule
//   U <- C R^-1 U~_K                                 (lift, second buffer)
// Randomized step (Eqs. 7-11 with q power iterations, ell = K + p < n):
//   X_0 = Omega;  q times: P = C^T C X, X = P chol(P^T P)^-1
//   final pass: P = C^T Y, G_Y = Y^T Y with Y = C X
//   R_Y = chol(G_Y), R_P = QR factor of P (Cholesky-QR2), R_b = R_P R_Y^-1,
//   U~, S from the Jacobi SVD of R_b^T (the left factor of B = Q^T C),
//   U <- C X R_Y^-1 U~_K.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"

using namespace psvd;

// ----------------------------------------------------------------------------
// Test matrix: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) keyed by the
// seed, counter (call index, batch); Box-Muller on two 53-bit uniforms.
// ----------------------------------------------------------------------------
namespace {

inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int rnd = 0; rnd < 10; ++rnd) {
        uint64_t a = (uint64_t)0xD2511F53u * c[0];
        uint64_t b = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t n0 = (uint32_t)(b >> 32) ^ c[1] ^ k0;
        uint32_t n1 = (uint32_t)b;
        uint32_t n2 = (uint32_t)(a >> 32) ^ c[3] ^ k1;
        uint32_t n3 = (uint32_t)a;
        c[0] = n0;
        c[1] = n1;
        c[2] = n2;
        c[3] = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

inline double bf16_round(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) != 0x7F800000u) u += 0x7FFFu + ((u >> 16) & 1u);
    u &= 0xFFFF0000u;
    float g;
    std::memcpy(&g, &u, 4);
    return (double)g;
}

// precision: 0 keep FP64, 1 round to FP32, 2 round to FP32 then BF16 (RNE).
void gen_omega(uint64_t seed, int64_t batch, int64_t n, int64_t l, int rounding, double* out) {
    const int64_t total = n * l;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int64_t t = 0; 2 * t < total; ++t) {
        uint32_t c[4] = {(uint32_t)t, (uint32_t)((uint64_t)t >> 32), (uint32_t)batch, (uint32_t)((uint64_t)batch >> 32)};
        philox10(c, k0, k1);
        const double s53 = 1.0 / 9007199254740992.0;
        double u1 = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6)) * s53;
        double u2 = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6)) * s53;
        double rad = std::sqrt(-2.0 * std::log(1.0 - u1));
        // cos and sin by separate C-library calls (never a merged sincos, whose
        // last bit may differ): the volatile argument prevents the merge.
        volatile double ang = 6.283185307179586476925286766559 * u2;
        double z[2] = {rad * std::cos(ang), rad * std::sin(ang)};
        for (int h = 0; h < 2 && 2 * t + h < total; ++h) {
            double v = z[h];
            if (rounding == 1) v = (double)(float)v;
            else if (rounding == 2) v = bf16_round((float)v);
            out[2 * t + h] = v;
        }
    }
}

int omega_rounding(int precision) { return precision == PSVD_PREC_FP64 ? 0 : (precision == PSVD_PREC_FP32 ? 1 : 2); }

const char* status_name(int s) {
    switch (s) {
        case PSVD_OK: return "PSVD_OK";
        case PSVD_E_INVAL: return "PSVD_E_INVAL";
        case PSVD_E_SHAPE: return "PSVD_E_SHAPE";
        case PSVD_E_DTYPE: return "PSVD_E_DTYPE";
        case PSVD_E_NOMEM: return "PSVD_E_NOMEM";
        case PSVD_E_NONFINITE: return "PSVD_E_NONFINITE";
        case PSVD_E_NOCONV: return "PSVD_E_NOCONV";
        case PSVD_E_BREAKDOWN: return "PSVD_E_BREAKDOWN";
        case PSVD_E_DEVICE: return "PSVD_E_DEVICE";
        case PSVD_E_STATE: return "PSVD_E_STATE";
        default: return "PSVD_E_UNKNOWN";
    }
}

// Device allocation that grows on demand.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t b) {
        if (b <= bytes) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, b);
        if (e == hipSuccess) bytes = b;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T* as() const { return (T*)p; }
};

PanelBlock make_block(const void* p, int64_t ld, int dtype, int ncols) {
    PanelBlock b;
    b.ptr = p;
    b.ld = ld;
    b.dtype = dtype;
    b.ncols = ncols;
    return b;
}

PanelSeg make_seg(int64_t rows) {
    PanelSeg s;
    std::memset(&s, 0, sizeof(s));
    s.rows = rows;
    return s;
}

void seg_add(PanelSeg& s, const PanelBlock& b) {
    if (b.ncols <= 0) return;
    s.blk[s.nblk++] = b;
    s.ncols += b.ncols;
}

int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace

// ----------------------------------------------------------------------------
// Handle.
// ----------------------------------------------------------------------------
struct psvd_handle {
    int64_t M = 0;
    int32_t K = 0;
    double ff = 1.0;
    int32_t p = 0, q = 0, ell = 0;
    psvd_options opt;
    hipStream_t stream = nullptr;
    int device = 0;

    int32_t r = 0;
    int64_t batch = 0;
    int32_t cur = 0;
    int32_t u_dtype = PSVD_F64;
    int64_t ldu = 0;
    DevBuf U[2];
    DevBuf s[2];        // K doubles each
    DevBuf d;           // K doubles: ff * s

    // workspace
    int32_t nmax = 0;   // panel width the workspace is sized for
    DevBuf part;        // k_tn partials (FP64)
    DevBuf partP;       // fused partials (FP32)
    DevBuf partG;       // fused G partials (FP64)
    DevBuf tall;        // M x max(n, ell) temporary (Q1 or Y)
    DevBuf small;       // small FP64 matrices
    DevBuf ivec;        // small int scratch
    DevBuf status;      // int32 x 2: status, sweeps
    int32_t* status_host = nullptr;  // pinned
    double* omega_host[2] = {nullptr, nullptr};  // pinned staging, alternating per update
    hipEvent_t omega_ev[2] = {nullptr, nullptr};
    size_t omega_host_cap = 0;

    psvd_stats_t stats;
    std::string err;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;

    // PSVD_OPT_PROFILE: event pairs around tall-panel launches, resolved at sync points.
    std::vector<hipEvent_t> prof_ev;
    std::vector<int> prof_pending;   // (class, event index) pairs, flattened
    int prof_next = 0;
};

static bool profiling(const psvd_handle* h) { return (h->opt.flags & PSVD_OPT_PROFILE) != 0; }

// Resolve the recorded event pairs (the stream must have passed them).
static void prof_resolve(psvd_handle* h) {
    for (size_t i = 0; i + 1 < h->prof_pending.size(); i += 2) {
        int cls = h->prof_pending[i], e = h->prof_pending[i + 1];
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->prof_ev[e], h->prof_ev[e + 1]) == hipSuccess) {
            h->stats.kernel_launches[cls] += 1;
            h->stats.kernel_ms[cls] += ms;
        }
    }
    h->prof_pending.clear();
    h->prof_next = 0;
}

static int prof_begin(psvd_handle* h, int cls) {
    if (!profiling(h)) return -1;
    if (h->prof_next + 2 > (int)h->prof_ev.size()) {
        (void)hipStreamSynchronize(h->stream);
        prof_resolve(h);
        if (h->prof_ev.size() < 512) {
            size_t old = h->prof_ev.size();
            h->prof_ev.resize(512);
            for (size_t i = old; i < h->prof_ev.size(); ++i) (void)hipEventCreate(&h->prof_ev[i]);
        }
    }
    int e = h->prof_next;
    h->prof_next += 2;
    (void)hipEventRecord(h->prof_ev[e], h->stream);
    h->prof_pending.push_back(cls);
    h->prof_pending.push_back(e);
    return e;
}

static void prof_end(psvd_handle* h, int e) {
    if (e >= 0) (void)hipEventRecord(h->prof_ev[e + 1], h->stream);
}

static int fail(psvd_handle* h, int code, const std::string& msg) {
    if (h) h->err = std::string(status_name(code)) + ": " + msg;
    return code;
}

static int hip_fail(psvd_handle* h, hipError_t e, const char* what) {
    return fail(h, e == hipErrorOutOfMemory ? PSVD_E_NOMEM : PSVD_E_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, expr)                                   \
    do {                                                  \
        hipError_t _e = (expr);                           \
        if (_e != hipSuccess) return hip_fail(h, _e, #expr); \
    } while (0)

// Small-matrix layout inside h->small (all FP64, column-major), sized for
// panel width n and sketch width l.
struct SmallLayout {
    double *G, *G2, *R1, *Ri, *Z, *T, *Xn, *sm_u, *vec;
    double *P, *P1, *X, *Om, *H, *H2, *RY, *RYi, *M2, *G_Y, *R1b;
    size_t total;
};

static SmallLayout small_layout(double* base, int n, int l, int K) {
    SmallLayout L;
    size_t off = 0;
    auto take = [&](size_t cnt) {
        double* p = base ? base + off : nullptr;
        off += (cnt + 31) & ~(size_t)31;
        return p;
    };
    size_t nn = (size_t)n * n, nl = (size_t)n * std::max(l, 1), ll = (size_t)std::max(l, 1) * std::max(l, 1);
    size_t nk = (size_t)std::max(n, l) * K;
    L.G = take(nn);
    L.G2 = take(nn);
    L.R1 = take(nn);
    L.Ri = take(nn);
    L.Z = take(nn);
    L.T = take(nk);
    L.Xn = take(nn);
    L.sm_u = take(nk);
    L.vec = take(4 * (size_t)std::max(n, l) + 64);
    L.P = take(nl);
    L.P1 = take(nl);
    L.X = take(nl);
    L.Om = take(nl);
    L.H = take(ll);
    L.H2 = take(ll);
    L.RY = take(ll);
    L.RYi = take(ll);
    L.M2 = take(ll);
    L.G_Y = take(ll);
    L.R1b = take(ll);
    L.total = off;
    return L;
}

static int ensure_workspace(psvd_handle* h, int n) {
    if (n <= h->nmax) return PSVD_OK;
    int l = h->ell;
    int w = std::max(n, l);
    SmallLayout L = small_layout(nullptr, n, l, h->K);
    HIPCHK(h, h->small.ensure(L.total * sizeof(double)));
    HIPCHK(h, h->ivec.ensure((size_t)(w + 64) * sizeof(int32_t)));
    // k_tn partials: items x output blocks stays near 1024 (see pick_chunk)
    int nb = ceil_div(w, 64);
    size_t nob = (size_t)nb * nb;
    HIPCHK(h, h->part.ensure((size_t)(2048 + 2 * nob) * 64 * 64 * sizeof(double)));
    int np = ((n + 15) / 16) * 16;
    int nlb = ceil_div(std::max(l, 1), 64);
    HIPCHK(h, h->partP.ensure((size_t)256 * nlb * np * 64 * sizeof(float)));
    HIPCHK(h, h->partG.ensure((size_t)256 * 64 * 64 * sizeof(double)));
    int esz = h->u_dtype == PSVD_F64 ? 8 : 4;
    // tall temporary: Q1 (M x n) for the deterministic step, Y (M x ell) otherwise
    int tall_cols = (l > 0 && l < n) ? l : n;
    HIPCHK(h, h->tall.ensure((size_t)h->M * tall_cols * esz));
    h->nmax = n;
    return PSVD_OK;
}

// ----------------------------------------------------------------------------
// Panel helpers (launch + fixed-order reduction into a dense FP64 result).
// ----------------------------------------------------------------------------
static int64_t pick_chunk(int64_t rows, int nob, int tm) {
    int64_t target = std::max<int64_t>(1, 1024 / std::max(1, nob));
    target = std::min<int64_t>(target, 1024);
    int64_t chunk = (rows + target - 1) / target;
    chunk = ((chunk + tm - 1) / tm) * tm;
    return std::max<int64_t>(chunk, tm);
}

// out (nl x nr FP64) = L^T R over all rows of the single-segment operands.
static int tn_product(psvd_handle* h, const PanelSeg& L, const PanelSeg& R, bool sym, bool fp64, double* out,
                      const double* row_scale, int nscale, const int32_t* skip, int skip_mask) {
    const int mbl = ceil_div(L.ncols, 64), mbr = ceil_div(R.ncols, 64);
    const int nob = sym ? mbl * (mbl + 1) / 2 : mbl * mbr;
    int64_t chunk = pick_chunk(L.rows, nob, 64);
    int nitems = ceil_div(L.rows, chunk);
    TnArgs a;
    std::memset(&a, 0, sizeof(a));
    a.lseg = L;
    a.rseg = R;
    a.chunk = chunk;
    a.mbl = mbl;
    a.sym = sym ? 1 : 0;
    a.part = h->part.as<double>();
    a.skip = skip;
    a.skip_mask = skip_mask;
    a.nob = nob;
    int pe = prof_begin(h, PSVD_KC_TN);
    HIPCHK(h, launch_tn(fp64, a, nitems, h->stream));
    prof_end(h, pe);
    TnReduceArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.row_scale = row_scale;
    ra.nscale = nscale;
    ra.part = h->part.as<double>();
    ra.seg_item0 = nullptr;
    ra.nitems = nitems;
    ra.mbl = mbl;
    ra.nob = nob;
    ra.nl = L.ncols;
    ra.nr = R.ncols;
    ra.sym = sym ? 1 : 0;
    ra.out = out;
    ra.skip = skip;
    ra.skip_mask = skip_mask;
    HIPCHK(h, launch_tn_reduce(ra, 1, h->stream));
    return PSVD_OK;
}

// out (rows x nx) = S X with X (S.ncols x nx, ld ldx) FP64.
static int nn_product(psvd_handle* h, const PanelSeg& S, const double* X, int64_t ldx, int nx, bool fp64,
                      const double* row_scale, int nscale, const int32_t* skip, int skip_mask,
                      int cls = PSVD_KC_NN, int need_mask = 0, int accumulate = 0) {
    int nbx = ceil_div(nx, 64);
    int64_t chunk = pick_chunk(S.rows, nbx, 64);
    int nitems = ceil_div(S.rows, chunk);
    NnArgs a;
    std::memset(&a, 0, sizeof(a));
    a.seg = S;
    a.chunk = chunk;
    a.row_scale = row_scale;
    a.nscale = nscale;
    a.X = X;
    a.ldx = ldx;
    a.n = S.ncols;
    a.nx = nx;
    a.skip = skip;
    a.skip_mask = skip_mask;
    a.need_mask = need_mask;
    a.accumulate = accumulate;
    int pe = prof_begin(h, cls);
    HIPCHK(h, launch_nn(fp64, a, nitems, h->stream));
    prof_end(h, pe);
    return PSVD_OK;
}

static PanelSeg small_seg(const double* p, int rows, int cols, int ld, double* out = nullptr, int ldo = 0) {
    PanelSeg s = make_seg(rows);
    seg_add(s, make_block(p, ld, PSVD_F64, cols));
    s.out = out;
    s.ldo = ldo;
    s.out_dtype = PSVD_F64;
    return s;
}

// X_new = orth(P) = P chol(P^T P)^-1 (P: n x l FP64), then rows scaled by D.
static int small_orth(psvd_handle* h, const SmallLayout& L, int n, int l, double* Xout, const int32_t* st) {
    PanelSeg Ps = small_seg(L.P, n, l, n);
    int rc = tn_product(h, Ps, Ps, true, true, L.H, nullptr, 0, nullptr, 0);
    if (rc) return rc;
    CholArgs ca;
    ca.H = L.H;
    ca.Ri = L.RYi;   // scratch R^-1
    ca.l = l;
    ca.status = (int32_t*)st;
    ca.flag_bit = DEV_FALLBACK;
    HIPCHK(h, launch_small_chol(ca, h->stream));
    Ps.out = Xout;
    Ps.ldo = n;
    rc = nn_product(h, Ps, L.RYi, l, l, true, h->d.as<double>(), h->r, nullptr, 0);
    return rc;
}

// ----------------------------------------------------------------------------
// C ABI.
// ----------------------------------------------------------------------------
extern "C" {

void psvd_default_options(psvd_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->method = PSVD_DETERMINISTIC;
    opt->precision = PSVD_PREC_FP64;
    opt->seed = 0;
    opt->stream = nullptr;
    opt->max_sweeps = 60;
    opt->flags = 0;
    opt->tile_rows = 0;
}

const char* psvd_status_string(int status) { return status_name(status); }

const char* psvd_last_error(const psvd_handle* h) { return h ? h->err.c_str() : "null handle"; }

int psvd_initialize(psvd_handle** out, int64_t M, int32_t K, double ff, int32_t oversampling, int32_t power_iters,
                    const psvd_options* opt) {
    if (!out) return PSVD_E_INVAL;
    *out = nullptr;
    psvd_options o;
    psvd_default_options(&o);
    if (opt) o = *opt;
    if (o.max_sweeps <= 0) o.max_sweeps = 60;
    if (M < 1 || K < 1 || K > M || !(ff > 0.0 && ff <= 1.0) || oversampling < 0 || power_iters < 0 ||
        (o.method != PSVD_DETERMINISTIC && o.method != PSVD_RANDOMIZED) ||
        (o.precision < PSVD_PREC_FP64 || o.precision > PSVD_PREC_MIXED))
        return PSVD_E_INVAL;
    psvd_handle* h = new (std::nothrow) psvd_handle();
    if (!h) return PSVD_E_NOMEM;
    h->M = M;
    h->K = K;
    h->ff = ff;
    h->p = oversampling;
    h->q = power_iters;
    h->ell = o.method == PSVD_RANDOMIZED ? K + oversampling : 0;
    h->opt = o;
    h->stream = (hipStream_t)o.stream;
    h->u_dtype = o.precision == PSVD_PREC_FP64 ? PSVD_F64 : PSVD_F32;
    h->ldu = ((M + 63) / 64) * 64;
    std::memset(&h->stats, 0, sizeof(h->stats));
    int esz = h->u_dtype == PSVD_F64 ? 8 : 4;
    hipError_t e = hipGetDevice(&h->device);
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        e = h->U[b].ensure((size_t)h->ldu * K * esz);
        if (e == hipSuccess) e = h->s[b].ensure((size_t)K * sizeof(double));
    }
    if (e == hipSuccess) e = h->d.ensure((size_t)K * sizeof(double));
    if (e == hipSuccess) e = h->status.ensure(64);
    if (e == hipSuccess) e = hipHostMalloc((void**)&h->status_host, 64, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreate(&h->ev0);
    if (e == hipSuccess) e = hipEventCreate(&h->ev1);
    if (e == hipSuccess) e = hipEventCreate(&h->omega_ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&h->omega_ev[1]);
    if (e == hipSuccess) e = hipMemsetAsync(h->U[0].p, 0, h->U[0].bytes, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->U[1].p, 0, h->U[1].bytes, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->s[0].p, 0, h->s[0].bytes, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->s[1].p, 0, h->s[1].bytes, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        psvd_finalize(h);
        return e == hipErrorOutOfMemory ? PSVD_E_NOMEM : PSVD_E_DEVICE;
    }
    *out = h;
    return PSVD_OK;
}

void psvd_finalize(psvd_handle* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    for (int b = 0; b < 2; ++b) {
        h->U[b].release();
        h->s[b].release();
    }
    h->d.release();
    h->part.release();
    h->partP.release();
    h->partG.release();
    h->tall.release();
    h->small.release();
    h->ivec.release();
    h->status.release();
    if (h->status_host) (void)hipHostFree(h->status_host);
    for (int b = 0; b < 2; ++b) {
        if (h->omega_host[b]) (void)hipHostFree(h->omega_host[b]);
        if (h->omega_ev[b]) (void)hipEventDestroy(h->omega_ev[b]);
    }
    for (hipEvent_t e : h->prof_ev) (void)hipEventDestroy(e);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    delete h;
}

int psvd_rank(const psvd_handle* h, int32_t* r) {
    if (!h || !r) return PSVD_E_INVAL;
    *r = h->r;
    return PSVD_OK;
}

int psvd_get_omega(const psvd_handle* h, int64_t batch, int64_t n, double* out) {
    if (!h || !out || batch < 0 || n < 1 || h->ell < 1) return PSVD_E_INVAL;
    gen_omega(h->opt.seed, batch, n, h->ell, omega_rounding(h->opt.precision), out);
    return PSVD_OK;
}

int psvd_stats(const psvd_handle* hc, psvd_stats_t* out) {
    psvd_handle* h = const_cast<psvd_handle*>(hc);
    if (!h || !out) return PSVD_E_INVAL;
    if (profiling(h)) {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        prof_resolve(h);
    }
    *out = h->stats;
    return PSVD_OK;
}

int psvd_reset_stats(psvd_handle* h) {
    if (!h) return PSVD_E_INVAL;
    if (profiling(h)) {
        HIPCHK(h, hipStreamSynchronize(h->stream));
        h->prof_pending.clear();
        h->prof_next = 0;
    }
    std::memset(&h->stats, 0, sizeof(h->stats));
    return PSVD_OK;
}

static int finish_status(psvd_handle* h, int32_t st) {
    if (st & DEV_NONFINITE) return fail(h, PSVD_E_NONFINITE, "non-finite values reached the small factorisation");
    if (st & DEV_BREAKDOWN) return fail(h, PSVD_E_BREAKDOWN, "Cholesky breakdown (fallback disabled)");
    if (st & DEV_NOCONV) return fail(h, PSVD_E_NOCONV, "Jacobi SVD did not converge within max_sweeps");
    return PSVD_OK;
}

int psvd_incorporate_data(psvd_handle* h, const void* A, int64_t M, int64_t N, int64_t lda, int32_t dtype) {
    if (!h) return PSVD_E_INVAL;
    h->err.clear();
    if (N < 0 || (N > 0 && !A)) return fail(h, PSVD_E_INVAL, "N < 0 or null data");
    if (M != h->M) return fail(h, PSVD_E_SHAPE, "row count differs from the handle's M");
    if (lda < M) return fail(h, PSVD_E_SHAPE, "lda < M");
    if (dtype != PSVD_F32 && dtype != PSVD_F64) return fail(h, PSVD_E_DTYPE, "unknown dtype");
    if (dtype == PSVD_F64 && h->u_dtype != PSVD_F64) return fail(h, PSVD_E_DTYPE, "FP64 data needs FP64 precision");
    if (N == 0) return PSVD_OK;
    if (N > 1 << 20) return fail(h, PSVD_E_SHAPE, "batch too wide");
    const int r = h->r;
    const int n = r + (int)N;
    if (n > M) return fail(h, PSVD_E_SHAPE, "panel wider than tall (r + N > M)");
    int rc = ensure_workspace(h, n);
    if (rc) return rc;
    const int prec = h->opt.precision;
    const bool fp64 = prec == PSVD_PREC_FP64;
    const bool randomized = h->ell > 0 && h->ell < n;
    const int l = randomized ? h->ell : 0;
    const int rk = randomized ? std::min(h->K, l) : std::min<int>(h->K, n);
    hipStream_t st = h->stream;
    SmallLayout L = small_layout(h->small.as<double>(), n, l, h->K);
    int32_t* dstat = h->status.as<int32_t>();
    int32_t* dsweeps = dstat + 1;
    const int cur = h->cur, nxt = 1 - cur;
    double* s_cur = h->s[cur].as<double>();
    double* s_new = h->s[nxt].as<double>();

    HIPCHK(h, hipEventRecord(h->ev0, st));
    HIPCHK(h, hipMemsetAsync(dstat, 0, 8, st));
    HIPCHK(h, launch_make_scale(h->d.as<double>(), s_cur, r, h->ff, st));

    // Panel [U | A] (unscaled) and its lift output.
    PanelSeg C = make_seg(M);
    if (r > 0) seg_add(C, make_block(h->U[cur].p, h->ldu, h->u_dtype, r));
    seg_add(C, make_block(A, lda, dtype, (int)N));
    C.out = h->U[nxt].p;
    C.ldo = h->ldu;
    C.out_dtype = h->u_dtype;
    const double* dsc = h->d.as<double>();
    const int tall_dtype = h->u_dtype;

    if (!randomized) {
        // ---- deterministic: Cholesky-QR2 + Jacobi SVD of R ----
        rc = tn_product(h, C, C, true, true, L.G, nullptr, 0, nullptr, 0);
        if (rc) return rc;
        SmallArgs sa;
        std::memset(&sa, 0, sizeof(sa));
        sa.n = n;
        sa.r = r;
        sa.K = h->K;
        sa.l = 0;
        sa.max_sweeps = h->opt.max_sweeps;
        sa.allow_fallback = (h->opt.flags & PSVD_OPT_NO_FALLBACK) ? 0 : 1;
        sa.d = dsc;
        sa.G = L.G;
        sa.G2 = L.G2;
        sa.R1 = L.R1;
        sa.Ri = L.Ri;
        sa.Z = L.Z;
        sa.T = L.T;
        sa.Xn = L.Xn;
        sa.s_out = s_new;
        sa.small_u = L.sm_u;
        sa.vec = L.vec;
        sa.ivec = h->ivec.as<int32_t>();
        sa.status = dstat;
        sa.sweeps = dsweeps;
        HIPCHK(h, launch_small_det1(sa, st));
        const int skipmask = DEV_FALLBACK | DEV_NONFINITE | DEV_BREAKDOWN;
        // Q1 = C D R1^-1 (tall temporary), G2 = Q1^T Q1.
        PanelSeg Q = C;
        Q.out = h->tall.p;
        Q.ldo = M;
        Q.out_dtype = tall_dtype;
        rc = nn_product(h, Q, L.Xn, n, n, fp64, nullptr, 0, dstat, skipmask);
        if (rc) return rc;
        PanelSeg Q1 = make_seg(M);
        seg_add(Q1, make_block(h->tall.p, M, tall_dtype, n));
        rc = tn_product(h, Q1, Q1, true, true, L.G2, nullptr, 0, dstat, skipmask);
        if (rc) return rc;
        HIPCHK(h, launch_small_det2(sa, st));
        // Lift: U = Q1 R2^-1 U~_rk from the kept Cholesky-QR factor; on the eigen
        // route (no Q1) U = C D V_rk diag(1/sigma) straight from the panel.
        PanelSeg Qs = Q1;
        Qs.out = h->U[nxt].p;
        Qs.ldo = h->ldu;
        Qs.out_dtype = h->u_dtype;
        rc = nn_product(h, Qs, L.T, n, rk, fp64, nullptr, 0, dstat, skipmask, PSVD_KC_LIFT);
        if (rc) return rc;
        rc = nn_product(h, C, L.T, n, rk, fp64, nullptr, 0, dstat, DEV_NONFINITE | DEV_BREAKDOWN, PSVD_KC_LIFT,
                        DEV_FALLBACK);
        if (rc) return rc;
    } else {
        // ---- randomized range finder ----
        size_t need = (size_t)n * l;
        const int ob = (int)(h->batch & 1);
        if (need > h->omega_host_cap) {
            HIPCHK(h, hipStreamSynchronize(st));
            for (int b = 0; b < 2; ++b) {
                if (h->omega_host[b]) (void)hipHostFree(h->omega_host[b]);
                h->omega_host[b] = nullptr;
            }
            h->omega_host_cap = 0;
            for (int b = 0; b < 2; ++b)
                HIPCHK(h, hipHostMalloc((void**)&h->omega_host[b], need * sizeof(double), hipHostMallocDefault));
            h->omega_host_cap = need;
        } else {
            // the update two batches back may still be copying from this buffer
            HIPCHK(h, hipEventSynchronize(h->omega_ev[ob]));
        }
        gen_omega(h->opt.seed, h->batch, n, l, omega_rounding(prec), h->omega_host[ob]);
        HIPCHK(h, hipMemcpyAsync(L.X, h->omega_host[ob], need * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(h, hipEventRecord(h->omega_ev[ob], st));
        // X' = D Omega
        HIPCHK(h, launch_scale_rows(L.X, n, l, n, dsc, r, 1, st));
        const int np = ((n + 15) / 16) * 16;
        const int nlb = ceil_div(l, 64);
        auto pass = [&](bool bf16, bool want_g) -> int {
            // P = D C'^T (C' X')  [+ G_Y = Y^T Y]
            bool fuse_ok = !fp64 && fused_fits(bf16, bf16 ? (np > 320 ? 16 : 32) : 32, np) && (!want_g || nlb == 1);
            if (fuse_ok) {
                FusedArgs fa;
                std::memset(&fa, 0, sizeof(fa));
                fa.seg = C;
                fa.X = L.X;
                fa.ldx = n;
                fa.n = n;
                fa.np = np;
                fa.lx = l;
                fa.nlb = nlb;
                fa.tm = bf16 ? (np > 320 ? 16 : 32) : 32;
                fa.nwg = 256;
                fa.tiles = (M + fa.tm - 1) / fa.tm;
                if (fa.tiles < fa.nwg) fa.nwg = (int)fa.tiles;
                fa.partP = h->partP.as<float>();
                fa.partG = h->partG.as<double>();
                fa.want_g = want_g ? 1 : 0;
                int pe = prof_begin(h, bf16 ? PSVD_KC_FUSED_BF16 : PSVD_KC_FUSED_F32);
                HIPCHK(h, launch_fused(bf16, fa, st));
                prof_end(h, pe);
                FusedReduceArgs ra;
                std::memset(&ra, 0, sizeof(ra));
                ra.row_scale = dsc;
                ra.nscale = r;
                ra.partP = h->partP.as<float>();
                ra.partG = h->partG.as<double>();
                ra.nwg = fa.nwg;
                ra.nlb = nlb;
                ra.np = np;
                ra.n = n;
                ra.lx = l;
                ra.want_g = fa.want_g;
                ra.P = L.P;
                ra.G = L.G_Y;
                HIPCHK(h, launch_fused_reduce(ra, st));
                return PSVD_OK;
            }
            // Unfused: Y = C X' (tall temporary), P = D C^T Y, G_Y = Y^T Y.
            PanelSeg Ys = C;
            Ys.out = h->tall.p;
            Ys.ldo = M;
            Ys.out_dtype = tall_dtype;
            int rc2 = nn_product(h, Ys, L.X, n, l, fp64, nullptr, 0, nullptr, 0);
            if (rc2) return rc2;
            PanelSeg Y = make_seg(M);
            seg_add(Y, make_block(h->tall.p, M, tall_dtype, l));
            rc2 = tn_product(h, C, Y, false, fp64, L.P, dsc, r, nullptr, 0);
            if (rc2) return rc2;
            if (want_g) rc2 = tn_product(h, Y, Y, true, true, L.G_Y, nullptr, 0, nullptr, 0);
            return rc2;
        };
        for (int it = 0; it < h->q; ++it) {
            rc = pass(prec == PSVD_PREC_MIXED, false);
            if (rc) return rc;
            rc = small_orth(h, L, n, l, L.X, dstat);   // X' = D orth(P)
            if (rc) return rc;
        }
        rc = pass(false, true);
        if (rc) return rc;
        // R_Y = chol(G_Y)
        CholArgs cy;
        cy.H = L.G_Y;
        cy.Ri = L.RYi;
        cy.l = l;
        cy.status = dstat;
        cy.flag_bit = DEV_FALLBACK;
        HIPCHK(h, launch_small_chol(cy, st));
        // R_P: Cholesky-QR2 of P.
        PanelSeg Ps = small_seg(L.P, n, l, n);
        rc = tn_product(h, Ps, Ps, true, true, L.H, nullptr, 0, nullptr, 0);
        if (rc) return rc;
        CholArgs c1;
        c1.H = L.H;          // -> R1
        c1.Ri = L.R1b;       // R1^-1
        c1.l = l;
        c1.status = dstat;
        c1.flag_bit = DEV_FALLBACK;
        HIPCHK(h, launch_small_chol(c1, st));
        Ps.out = L.P1;
        Ps.ldo = n;
        rc = nn_product(h, Ps, L.R1b, l, l, true, nullptr, 0, nullptr, 0);
        if (rc) return rc;
        PanelSeg P1s = small_seg(L.P1, n, l, n);
        rc = tn_product(h, P1s, P1s, true, true, L.H2, nullptr, 0, nullptr, 0);
        if (rc) return rc;
        RandFinalArgs rf;
        rf.l = l;
        rf.K = h->K;
        rf.max_sweeps = h->opt.max_sweeps;
        rf.RY = L.G_Y;
        rf.RYi = L.RYi;
        rf.R1 = L.H;
        rf.H2 = L.H2;
        rf.Z = L.Z;
        rf.M2 = L.M2;
        rf.s_out = s_new;
        rf.small_u = L.sm_u;
        rf.vec = L.vec;
        rf.ivec = h->ivec.as<int32_t>();
        rf.status = dstat;
        rf.sweeps = dsweeps;
        HIPCHK(h, launch_small_rand_final(rf, st));
        // T' = X' M2 (n x rk), U_new = C' T'.
        PanelSeg Xs = small_seg(L.X, n, l, n, L.T, n);
        rc = nn_product(h, Xs, L.M2, l, rk, true, nullptr, 0, nullptr, 0);
        if (rc) return rc;
        rc = nn_product(h, C, L.T, n, rk, fp64, nullptr, 0, dstat, DEV_NONFINITE | DEV_BREAKDOWN, PSVD_KC_LIFT);
        if (rc) return rc;
    }
    HIPCHK(h, hipEventRecord(h->ev1, st));
    const int prev_r = h->r;
    const int64_t prev_batch = h->batch;
    h->cur = nxt;
    h->r = rk;
    h->batch += 1;
    h->stats.batches += 1;
    h->stats.last_path = randomized ? 1 : 0;
    if (!(h->opt.flags & PSVD_OPT_ASYNC)) {
        hipError_t e = hipMemcpyAsync(h->status_host, dstat, 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            h->cur = cur;
            h->r = prev_r;
            h->batch = prev_batch;
            h->stats.batches -= 1;
            return hip_fail(h, e, "update");
        }
        int32_t sv = h->status_host[0];
        if (profiling(h)) prof_resolve(h);
        h->stats.last_sweeps = h->status_host[1];
        if (sv & DEV_FALLBACK) h->stats.fallbacks += 1;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) h->stats.last_update_ms = ms;
        int code = finish_status(h, sv);
        if (code != PSVD_OK) {
            h->cur = cur;
            h->r = prev_r;
            h->batch = prev_batch;
            h->stats.batches -= 1;
            return code;
        }
    }
    return PSVD_OK;
}

int psvd_singular_values(const psvd_handle* hc, double* out, int32_t cap, int32_t* r) {
    psvd_handle* h = const_cast<psvd_handle*>(hc);
    if (!h) return PSVD_E_INVAL;
    if (r) *r = h->r;
    if (h->r == 0) return PSVD_OK;
    if (!out || cap < h->r) return fail(h, PSVD_E_INVAL, "output capacity below the rank");
    HIPCHK(h, hipMemcpyAsync(out, h->s[h->cur].p, (size_t)h->r * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return PSVD_OK;
}

int psvd_modes_ptr(const psvd_handle* h, const void** U, int64_t* ldu, int32_t* dtype) {
    if (!h || !U) return PSVD_E_INVAL;
    *U = h->U[h->cur].p;
    if (ldu) *ldu = h->ldu;
    if (dtype) *dtype = h->u_dtype;
    return PSVD_OK;
}

int psvd_modes(const psvd_handle* hc, void* U, int64_t ldu, int32_t dtype) {
    psvd_handle* h = const_cast<psvd_handle*>(hc);
    if (!h || (!U && h->r > 0)) return PSVD_E_INVAL;
    if (ldu < h->M) return fail(h, PSVD_E_SHAPE, "ldu < M");
    if (dtype != PSVD_F32 && dtype != PSVD_F64) return fail(h, PSVD_E_DTYPE, "unknown dtype");
    if (h->r == 0) return PSVD_OK;
    if (dtype == h->u_dtype) {
        int esz = dtype == PSVD_F64 ? 8 : 4;
        HIPCHK(h, hipMemcpy2DAsync(U, ldu * esz, h->U[h->cur].p, h->ldu * esz, h->M * esz, h->r,
                                   hipMemcpyDeviceToDevice, h->stream));
        return PSVD_OK;
    }
    // conversion through the lift kernel with an identity operand
    std::vector<double> I((size_t)h->r * h->r, 0.0);
    for (int j = 0; j < h->r; ++j) I[(size_t)j * h->r + j] = 1.0;
    DevBuf tmp;
    HIPCHK(h, tmp.ensure(I.size() * sizeof(double)));
    HIPCHK(h, hipMemcpyAsync(tmp.p, I.data(), I.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
    PanelSeg S = make_seg(h->M);
    seg_add(S, make_block(h->U[h->cur].p, h->ldu, h->u_dtype, h->r));
    S.out = U;
    S.ldo = ldu;
    S.out_dtype = dtype;
    int rc = nn_product(h, S, tmp.as<double>(), h->r, h->r, true, nullptr, 0, nullptr, 0);
    HIPCHK(h, hipStreamSynchronize(h->stream));
    tmp.release();
    return rc;
}

}  // extern "C"
