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
#include <thread>
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
// Pairs [t0, t1) of the n x l matrix (entry 2 t + h from counter t).
void gen_omega_range(uint64_t seed, int64_t batch, int64_t total, int rounding, double* out, int64_t t0, int64_t t1) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int64_t t = t0; t < t1; ++t) {
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

// Every entry depends only on its own counter, so the pairs are split over a
// few host threads (the result does not depend on the split).
void gen_omega(uint64_t seed, int64_t batch, int64_t n, int64_t l, int rounding, double* out) {
    const int64_t total = n * l, pairs = (total + 1) / 2;
    const int64_t per = 2048;   // pairs per thread (~0.15 ms of work)
    int nt = (int)std::min<int64_t>(8, (pairs + per - 1) / per);
    if (nt <= 1) {
        gen_omega_range(seed, batch, total, rounding, out, 0, pairs);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (pairs + nt - 1) / nt;
    for (int i = 1; i < nt; ++i) {
        const int64_t t0 = i * chunk, t1 = std::min<int64_t>(pairs, t0 + chunk);
        if (t0 < t1) th.emplace_back(gen_omega_range, seed, batch, total, rounding, out, t0, t1);
    }
    gen_omega_range(seed, batch, total, rounding, out, 0, std::min<int64_t>(pairs, chunk));
    for (auto& x : th) x.join();
}

// Test-matrix entries: FP64 as drawn, FP32, or BF16 (the mixed and BF16 precisions).
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

// Device allocation that grows on demand.  A borrowed buffer (a region of
// memory the handle does not own) never allocates or frees: a request beyond
// its size fails with hipErrorOutOfMemory.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool borrowed = false;
    void borrow(void* q, size_t b) {
        p = q;
        bytes = b;
        borrowed = true;
    }
    hipError_t ensure(size_t b) {
        if (b <= bytes) return hipSuccess;
        if (borrowed) return hipErrorOutOfMemory;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, b);
        if (e == hipSuccess) bytes = b;
        return e;
    }
    void release() {
        if (p && !borrowed) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        borrowed = false;
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
    hipEvent_t omega_ev[2] = {nullptr, nullptr};  // upload of buffer b done (copy stream)
    hipEvent_t omega_used[2] = {nullptr, nullptr};  // device buffer b read by its update (main stream)
    DevBuf omega_dev[2];                          // device copies, alternating per update
    hipStream_t cstream = nullptr;                // uploads of the test matrix
    hipStream_t gstream = nullptr;                // captures a randomized update (never runs work)
    size_t omega_host_cap = 0;

    psvd_stats_t stats;
    int32_t async_fallbacks_seen = 0;
    std::string err;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipGraphExec_t rgraph = nullptr;              // the last randomized update's launches (captured)

    // PSVD_OPT_PROFILE: event pairs around tall-panel launches, resolved at sync points.
    std::vector<hipEvent_t> prof_ev;
    std::vector<int> prof_pending;   // (class, event index) pairs, flattened
    int prof_next = 0;

    // Partitioned streaming (psvd_pstream_*): row counts of the partitions and
    // their first row; the state U holds partition i's M_i x K block at element
    // offset poff[i] * K with leading dimension M_i.  Empty: one M-row panel.
    std::vector<int64_t> parts, poff;
    int32_t r_local = 0;
    DevBuf pdesc;       // partition panels and row-chunk work lists of one update
    DevBuf lrwork, lrom;   // low-rank SVD of the combined R: scratch, test matrix
};

static bool profiling(const psvd_handle* h) { return (h->opt.flags & PSVD_OPT_PROFILE) != 0; }

static int handle_omega_rounding(const psvd_handle* h) {
    return (h->opt.flags & PSVD_OPT_OMEGA_BF16) ? 2 : omega_rounding(h->opt.precision);
}

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

// Last error of a call without a handle (psvd_rsvd), per host thread.
static thread_local std::string g_call_err;

static int fail(psvd_handle* h, int code, const std::string& msg) {
    if (h) h->err = std::string(status_name(code)) + ": " + msg;
    return code;
}

static int hip_fail(psvd_handle* h, hipError_t e, const char* what) {
    return fail(h, e == hipErrorOutOfMemory ? PSVD_E_NOMEM : PSVD_E_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

static int sync_async(psvd_handle* h);

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

// Work items of the generic tall products (times output blocks).
static int split_items(const psvd_handle* h) { return h->opt.split_m > 0 ? h->opt.split_m : 1024; }
// Width the fused passes are planned for (at least the panel's).
static int plan_width(const psvd_handle* h, int n) { return std::max(n, (int)h->opt.panel_width); }

// Work-groups of a fused pass: wg_per_cu per compute unit (256 CUs), at most one per tile.
// The lift has no partial sums; by default it runs as many work-groups per CU
// as its LDS allows (up to 4), so more tile loads are in flight.
static int fused_wgs(const psvd_handle* h, int64_t tiles, size_t lift_lds = 0) {
    int per_cu = h->opt.wg_per_cu > 0 ? h->opt.wg_per_cu : 1;
    if (h->opt.wg_per_cu == 0 && lift_lds > 0) per_cu = (int)std::max<size_t>(1, std::min<size_t>(4, (160 * 1024) / lift_lds));
    const int64_t nwg = std::min<int64_t>((int64_t)256 * per_cu, FU_MAX_WG);
    return (int)std::max<int64_t>(1, std::min<int64_t>(nwg, tiles));
}

static int ensure_workspace(psvd_handle* h, int n) {
    if (n <= h->nmax) return PSVD_OK;
    int l = h->ell;
    int w = std::max(n, l);
    SmallLayout L = small_layout(nullptr, n, l, h->K);
    HIPCHK(h, h->small.ensure(L.total * sizeof(double)));
    HIPCHK(h, h->ivec.ensure((size_t)(3 * w + 64) * sizeof(int32_t)));
    // k_tn partials: items x output blocks stays near 1024 (see pick_chunk)
    int nb = ceil_div(w, 64);
    size_t nob = (size_t)nb * nb;
    // k_tn_x: one partial slot per row share, 256 work-groups over the
    // 320-column parts of a wide panel
    const size_t xblocks = (size_t)(256 / ceil_div(n, TNX_LCOLS)) * ceil_div(n, 64) * ceil_div(std::min(l, TNX_RCOLS), 64);
    HIPCHK(h, h->part.ensure(std::max((size_t)(2 * std::max(1024, split_items(h)) + 2 * nob), xblocks) * 64 * 64 *
                             sizeof(double)));
    // fused-pass partials: one NP x 64 block per (work-group, column block)
    const int pw = plan_width(h, n);
    int np = ((pw + 63) / 64) * 64;
    FusedPlan sp;
    for (int tr : {0, 32})
        if (sketch_plan(pw, tr, &sp)) np = std::max(np, sp.np);
    if (fused_plan(pw, h->opt.tile_rows, &sp)) np = std::max(np, sp.np);
    if (split_plan(pw, &sp)) np = std::max(np, sp.np);
    int nlb = ceil_div(std::max(l, 1), 64);
    const size_t wgs = (size_t)fused_wgs(h, INT64_MAX);
    HIPCHK(h, h->partP.ensure(wgs * nlb * np * 64 * sizeof(float)));
    HIPCHK(h, h->partG.ensure(wgs * 64 * 64 * sizeof(double)));
    h->nmax = n;
    return PSVD_OK;
}

// ----------------------------------------------------------------------------
// Panel helpers (launch + fixed-order reduction into a dense FP64 result).
// ----------------------------------------------------------------------------
// float4 loads need 16-byte aligned column starts: rows % 4 == 0 and every
// leading dimension a multiple of 4 with a 16-byte aligned base.
static bool seg_vec_ok(const PanelSeg& S, bool check_out) {
    if (S.rows % 4) return false;
    for (int b = 0; b < S.nblk; ++b)
        if ((S.blk[b].ld % 4) || ((uintptr_t)S.blk[b].ptr & 15)) return false;
    if (check_out && ((S.ldo % 4) || ((uintptr_t)S.out & 15))) return false;
    return true;
}

static bool seg_all_f32(const PanelSeg& S) {
    for (int b = 0; b < S.nblk; ++b)
        if (S.blk[b].dtype != PSVD_F32) return false;
    return true;
}

// The dtype of every block of S, or 0 when the blocks differ.
static int seg_dtype_all(const PanelSeg& S) {
    int d = S.nblk > 0 ? S.blk[0].dtype : 0;
    for (int b = 1; b < S.nblk; ++b)
        if (S.blk[b].dtype != d) d = 0;
    return d;
}

static int64_t pick_chunk(int64_t rows, int nob, int tm, int items = 1024) {
    int64_t target = std::max<int64_t>(1, items / std::max(1, nob));
    target = std::min<int64_t>(target, items);
    int64_t chunk = (rows + target - 1) / target;
    chunk = ((chunk + tm - 1) / tm) * tm;
    return std::max<int64_t>(chunk, tm);
}

// Row chunk of a TN product: k_tn and k_tn_v run one work-group per (item,
// output block), about `items` in all; k_tn_w (a Gram of 65..128 columns of
// one dtype) one per item and one per CU, so it takes at most 256 items.
static bool tn_wide(bool sym, int mbl, int dtype_all) { return sym && mbl == 2 && dtype_all != 0; }
constexpr int TN_WIDE_ITEMS = 256;
static int64_t tn_chunk(int64_t rows, int nob, bool wide, int items) {
    return wide ? chunk_for_items(&rows, 1, TN_WIDE_ITEMS) : pick_chunk(rows, nob, 64, items);
}

// out (nl x nr FP64) = L^T R over all rows of the single-segment operands.
static int tn_product(psvd_handle* h, const PanelSeg& L, const PanelSeg& R, bool sym, bool fp64, double* out,
                      const double* row_scale, int nscale, const int32_t* skip, int skip_mask) {
    const int mbl = ceil_div(L.ncols, 64), mbr = ceil_div(R.ncols, 64);
    const int nob = sym ? mbl * (mbl + 1) / 2 : mbl * mbr;
    const bool vec = seg_vec_ok(L, false) && seg_vec_ok(R, false);
    const int dt = seg_dtype_all(L) == seg_dtype_all(R) ? seg_dtype_all(L) : 0;
    int64_t chunk = tn_chunk(L.rows, nob, tn_wide(sym, mbl, dt), split_items(h));
    int nitems = ceil_div(L.rows, chunk);
    // wide FP32 projections (C^T Y of panels wider than the fused passes take):
    // one read of each operand, a partial slot per row share (k_tn_x), as many
    // shares as fill the CUs and the partial buffer holds
    int64_t xslots = 0;
    if (!sym && !fp64 && vec && dt == PSVD_F32 && L.ncols >= 128 && R.ncols > 32 && R.ncols <= TNX_RCOLS) {
        const int64_t nparts = ceil_div(L.ncols, TNX_LCOLS);
        const int64_t cap = (int64_t)(h->part.bytes / (64 * 64 * sizeof(double))) / nob;
        xslots = std::min<int64_t>(std::max<int64_t>(1, 256 / nparts), cap);
        if (xslots >= 1) {
            chunk = (int64_t)ceil_div(ceil_div(L.rows, xslots), 64) * 64;
            nitems = ceil_div(L.rows, chunk);
        }
    }
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
    a.vec = vec ? 1 : 0;
    a.dtype_all = dt;
    int pe = prof_begin(h, xslots >= 1 ? PSVD_KC_WIDE : PSVD_KC_TN);
    if (xslots >= 1) HIPCHK(h, launch_tn_x(a, nitems, h->stream));
    else HIPCHK(h, launch_tn(fp64, a, nitems, h->stream));
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
    int64_t chunk = pick_chunk(S.rows, nbx, 64, split_items(h));
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
    a.all_f32 = (!fp64 && seg_all_f32(S)) ? 1 : 0;
    a.vec_f32 = (a.all_f32 && seg_vec_ok(S, false)) ? 1 : 0;
    a.vec16 = seg_vec_ok(S, false) ? 1 : 0;
    if (cls == PSVD_KC_NN && nn_wide(fp64, a)) cls = PSVD_KC_WIDE;   // k_nn_x
    int pe = prof_begin(h, cls);
    HIPCHK(h, launch_nn(fp64, a, nitems, h->stream));
    prof_end(h, pe);
    return PSVD_OK;
}



// out (S.out) = S T with T (S.ncols x nx FP64): fused FP32 lift when the panel
// is FP32 and fits, otherwise the generic product.
static int lift_product(psvd_handle* h, const PanelSeg& S, const double* T, int64_t ldt, int nx, bool fp64,
                        const int32_t* skip, int skip_mask, int need_mask) {
    FusedPlan fp;
    if (!fp64 && seg_all_f32(S) && S.out_dtype == PSVD_F32 && skip == nullptr &&
        fused_plan(S.ncols, h->opt.tile_rows, &fp, true)) {
        FusedArgs fa;
        std::memset(&fa, 0, sizeof(fa));
        fa.seg = S;
        fa.X = T;
        fa.ldx = ldt;
        fa.n = S.ncols;
        fa.np = fp.np;
        fa.lx = nx;
        fa.nlb = ceil_div(nx, 64);
        fa.tm = fp.tm;
        fa.tiles = (S.rows + fp.tm - 1) / fp.tm;
        fa.nwg = fused_wgs(h, fa.tiles, fp.lds);
        fa.vec = seg_vec_ok(S, true) ? 1 : 0;
        int pe = prof_begin(h, PSVD_KC_LIFT);
        HIPCHK(h, launch_fused(2, fa, h->stream));
        prof_end(h, pe);
        return PSVD_OK;
    }
    return nn_product(h, S, T, ldt, nx, fp64, nullptr, 0, skip, skip_mask, PSVD_KC_LIFT, need_mask);
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
static int small_orth(psvd_handle* h, const SmallLayout& L, int n, int l, double* Xout, int32_t* st) {
    OrthArgs oa;
    std::memset(&oa, 0, sizeof(oa));
    oa.n = n;
    oa.l = l;
    oa.P = L.P;
    oa.G = L.H;
    oa.R = L.H2;
    oa.Ri = L.RYi;
    oa.vec = L.vec;
    oa.X = Xout;
    oa.d = h->d.as<double>();
    oa.r = h->r;
    oa.status = st;
    oa.flag_bit = DEV_FALLBACK;
    int pes = prof_begin(h, PSVD_KC_SMALL);
    HIPCHK(h, launch_small_orth(oa, h->stream));
    prof_end(h, pes);
    return PSVD_OK;
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

const char* psvd_last_error(const psvd_handle* h) { return h ? h->err.c_str() : g_call_err.c_str(); }

static bool tuning_ok(int32_t tile_rows, int32_t wg_per_cu, int32_t panel_width, int32_t split_m) {
    return (tile_rows == 0 || tile_rows == 16 || tile_rows == 32 || tile_rows == 64) && wg_per_cu >= 0 &&
           wg_per_cu <= FU_MAX_WG / 256 && panel_width >= 0 && panel_width <= 640 && split_m >= 0 &&
           split_m <= 8192 && (split_m == 0 || split_m >= 8);
}

int psvd_set_tuning(psvd_handle* h, int32_t tile_rows, int32_t wg_per_cu, int32_t panel_width, int32_t split_m) {
    if (!h || !tuning_ok(tile_rows, wg_per_cu, panel_width, split_m)) return PSVD_E_INVAL;
    if (int rc = sync_async(h)) return rc;
    HIPCHK(h, hipStreamSynchronize(h->stream));   // no update in flight uses the workspace
    h->opt.tile_rows = tile_rows;
    h->opt.wg_per_cu = wg_per_cu;
    h->opt.panel_width = panel_width;
    h->opt.split_m = split_m;
    h->nmax = 0;   // the workspace is re-sized for the new plans at the next update
    return PSVD_OK;
}

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
        (o.precision < PSVD_PREC_FP64 || o.precision > PSVD_PREC_BF16) ||
        !tuning_ok(o.tile_rows, o.wg_per_cu, o.panel_width, o.split_m))
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
    if (e == hipSuccess) e = hipMemset(h->status.p, 0, 64);
    if (e == hipSuccess) e = hipHostMalloc((void**)&h->status_host, 64, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreate(&h->ev0);
    if (e == hipSuccess) e = hipEventCreate(&h->ev1);
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        e = hipEventCreateWithFlags(&h->omega_ev[b], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->omega_used[b], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->cstream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking);
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
    h->pdesc.release();
    h->lrwork.release();
    h->lrom.release();
    h->partP.release();
    h->partG.release();
    h->tall.release();
    h->small.release();
    h->ivec.release();
    h->status.release();
    if (h->status_host) (void)hipHostFree(h->status_host);
    if (h->cstream) {
        (void)hipStreamSynchronize(h->cstream);
        (void)hipStreamDestroy(h->cstream);
    }
    if (h->gstream) (void)hipStreamDestroy(h->gstream);
    for (int b = 0; b < 2; ++b) {
        if (h->omega_host[b]) (void)hipHostFree(h->omega_host[b]);
        if (h->omega_ev[b]) (void)hipEventDestroy(h->omega_ev[b]);
        if (h->omega_used[b]) (void)hipEventDestroy(h->omega_used[b]);
        h->omega_dev[b].release();
    }
    for (hipEvent_t e : h->prof_ev) (void)hipEventDestroy(e);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->rgraph) (void)hipGraphExecDestroy(h->rgraph);
    delete h;
}

int psvd_rank(const psvd_handle* h, int32_t* r) {
    if (!h || !r) return PSVD_E_INVAL;
    *r = h->r;
    return PSVD_OK;
}

int psvd_get_omega(const psvd_handle* h, int64_t batch, int64_t n, double* out) {
    if (!h || !out || batch < 0 || n < 1 || h->ell < 1) return PSVD_E_INVAL;
    gen_omega(h->opt.seed, batch, n, h->ell, handle_omega_rounding(h), out);
    return PSVD_OK;
}

int psvd_stats(const psvd_handle* hc, psvd_stats_t* out) {
    psvd_handle* h = const_cast<psvd_handle*>(hc);
    if (!h || !out) return PSVD_E_INVAL;
    if (int rc = sync_async(h)) return rc;
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

// Synchronising calls of an asynchronous handle: wait for the stream, take the
// folded status of the updates since the last such call, and report the first
// device error (the state then holds the results of the failed update).
static int sync_async(psvd_handle* h) {
    if (!(h->opt.flags & PSVD_OPT_ASYNC)) return PSVD_OK;
    int32_t* dstat = h->status.as<int32_t>();
    HIPCHK(h, hipMemcpyAsync(h->status_host, dstat, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const int32_t sticky = h->status_host[2];
    h->stats.last_sweeps = h->status_host[3];
    h->stats.fallbacks += h->status_host[4] - h->async_fallbacks_seen;
    h->async_fallbacks_seen = h->status_host[4];
    if (sticky) {
        HIPCHK(h, hipMemsetAsync(dstat + 2, 0, sizeof(int32_t), h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        return finish_status(h, sticky);
    }
    return PSVD_OK;
}

int psvd_incorporate_data(psvd_handle* h, const void* A, int64_t M, int64_t N, int64_t lda, int32_t dtype) {
    if (!h) return PSVD_E_INVAL;
    h->err.clear();
    if (!h->parts.empty()) return fail(h, PSVD_E_STATE, "partitioned handle: use psvd_pstream_incorporate");
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
    // tall temporary: Q1 (M x n) for the deterministic step, Y (M x ell) otherwise
    {
        const int cols = (h->ell > 0 && h->ell < n) ? h->ell : n;
        HIPCHK(h, h->tall.ensure((size_t)M * cols * (h->u_dtype == PSVD_F64 ? 8 : 4)));
    }
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

    if (h->ev0) HIPCHK(h, hipEventRecord(h->ev0, st));
    if (!randomized) {   // status cleared and d = ff s (the randomized start does this in k_rand_begin)
        HIPCHK(h, launch_make_scale(dstat, h->d.as<double>(), s_cur, r, h->ff, st));
    }

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
        sa.stop_cos2 = h->opt.precision == PSVD_PREC_FP64 ? 0.0 : 0x1p-30;
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
        {
            int pes = prof_begin(h, PSVD_KC_SMALL_SVD);
            HIPCHK(h, launch_small_det1(sa, st));
            prof_end(h, pes);
        }
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
        {
            int pes = prof_begin(h, PSVD_KC_SMALL_SVD);
            HIPCHK(h, launch_small_det2(sa, st));
            prof_end(h, pes);
        }
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
        // Omega is generated on the host (the published Philox4x32-10 / Box-Muller
        // definition, bit-identical to the reference generator) and uploaded on
        // a copy stream into one of two device buffers, so the copy overlaps the
        // previous update; the main stream waits for it before k_rand_begin.
        size_t need = (size_t)n * l;
        const int ob = h->cstream ? (int)(h->batch & 1) : 0;
        if (!h->cstream) {
            // a handle without a copy stream (the allocation-free entry point): the
            // test matrix is generated into its fixed host buffer on this thread and
            // uploaded on the main stream
            if (need > h->omega_host_cap || need * sizeof(double) > h->omega_dev[0].bytes)
                return fail(h, PSVD_E_NOMEM, "test matrix larger than its fixed buffers");
            gen_omega_range(h->opt.seed, h->batch, (int64_t)need, handle_omega_rounding(h), h->omega_host[0], 0,
                            ((int64_t)need + 1) / 2);
            HIPCHK(h, hipMemcpyAsync(h->omega_dev[0].p, h->omega_host[0], need * sizeof(double), hipMemcpyHostToDevice,
                                     st));
        } else {
            if (need > h->omega_host_cap) {
                HIPCHK(h, hipStreamSynchronize(st));
                HIPCHK(h, hipStreamSynchronize(h->cstream));
                for (int b = 0; b < 2; ++b) {
                    if (h->omega_host[b]) (void)hipHostFree(h->omega_host[b]);
                    h->omega_host[b] = nullptr;
                }
                h->omega_host_cap = 0;
                for (int b = 0; b < 2; ++b) {
                    HIPCHK(h, hipHostMalloc((void**)&h->omega_host[b], need * sizeof(double), hipHostMallocDefault));
                    HIPCHK(h, h->omega_dev[b].ensure(need * sizeof(double)));
                }
                h->omega_host_cap = need;
            } else {
                // the upload two batches back may still be reading this host buffer
                HIPCHK(h, hipEventSynchronize(h->omega_ev[ob]));
            }
            gen_omega(h->opt.seed, h->batch, n, l, handle_omega_rounding(h), h->omega_host[ob]);
            // the device buffer is free once the update two batches back has read it
            HIPCHK(h, hipStreamWaitEvent(h->cstream, h->omega_used[ob], 0));
            HIPCHK(h, hipMemcpyAsync(h->omega_dev[ob].p, h->omega_host[ob], need * sizeof(double),
                                     hipMemcpyHostToDevice, h->cstream));
            HIPCHK(h, hipEventRecord(h->omega_ev[ob], h->cstream));
            HIPCHK(h, hipStreamWaitEvent(st, h->omega_ev[ob], 0));
        }
        // The launches of the range finder, lift included.  In the graph form
        // (PSVD_OPT_GRAPH) they are captured into one hipGraph (the test-matrix
        // upload and its wait stay outside) and launched as one, the executable
        // graph updated in place when only the arguments changed (new batch, the
        // other state buffers).
        auto enqueue = [&]() -> int {
            // status cleared, d = ff s, X' = D Omega
            HIPCHK(h, launch_rand_begin(dstat, h->d.as<double>(), s_cur, r, h->ff, L.X, h->omega_dev[ob].as<double>(), n,
                                        l, st));
            const int nlb = ceil_div(l, 64);
            // Fused passes, one read of the panel each: P = D C'^T (C' X') and, in
            // the final pass, the kept Y = C' X' and G_Y = Y^T Y.
            //   mixed: power passes on the BF16 matrix cores with every operand
            //          split into three BF16 terms, six term products: FP32-accurate
            //          (k_splitpass<., 3>); the final pass with pair splits
            //          (k_split64), G_Y from the kept Y
            //          (k_gram_kept); FP32 matrix cores (k_fused) on panels those
            //          kernels do not take.  (Pairs carry about 2^-17 relative error
            //          per operand; in the power iterations that error reaches the
            //          tail of the sketch amplified by (s_1 / s_j)^2, so those passes
            //          take the three-term split.)
            //   bf16:  power passes on plain BF16 operands (k_sketch_bf16), the final
            //          pass split-BF16 with a BF16-rounded test matrix (k_final_split)
            //   fp32:  FP32 matrix cores (k_fused);  fp64: the generic products
            enum { UNFUSED, SPLIT64, SKETCH_BF16, FINAL_SPLIT, FUSED_F32, SPLIT3 };
            auto pass = [&](bool final_pass) -> int {
                FusedPlan fp;
                int kind = UNFUSED;
                const bool vec = seg_vec_ok(C, false);
                const int pw = plan_width(h, n);
                if (!fp64 && seg_all_f32(C)) {
                    const bool mixed1 = prec == PSVD_PREC_MIXED && nlb == 1 && vec && M >= 4;
                    if (mixed1 && !final_pass && splitpass_plan(pw, 3, &fp))
                        kind = SPLIT3;
                    else if (mixed1 && final_pass && split64_plan(pw, &fp))
                        kind = SPLIT64;
                    else if (prec == PSVD_PREC_BF16 && !final_pass && sketch_plan(pw, h->opt.tile_rows, &fp))
                        kind = SKETCH_BF16;
                    else if (prec == PSVD_PREC_BF16 && final_pass && nlb == 1 && split_plan(pw, &fp)) kind = FINAL_SPLIT;
                    else if ((!final_pass || nlb == 1) && fused_plan(pw, h->opt.tile_rows, &fp)) kind = FUSED_F32;
                }
                if (kind != UNFUSED) {
                    FusedArgs fa;
                    std::memset(&fa, 0, sizeof(fa));
                    fa.seg = C;
                    fa.X = L.X;
                    fa.ldx = n;
                    fa.n = n;
                    fa.np = fp.np;
                    fa.lx = l;
                    fa.nlb = nlb;
                    fa.tm = fp.tm;
                    fa.tiles = (M + fa.tm - 1) / fa.tm;
                    fa.nwg = fused_wgs(h, fa.tiles);
                    fa.partP = h->partP.as<float>();
                    fa.partG = h->partG.as<double>();
                    const bool kept_gram = kind == SPLIT64;   // G_Y from the kept Y
                    fa.want_g = (final_pass && !kept_gram) ? 1 : 0;
                    fa.vec = vec ? 1 : 0;
                    if (final_pass) {   // keep Y = C X for the lift (U = Y R_Y^-1 U~_K)
                        fa.yout = h->tall.as<float>();
                        fa.ldy = M;
                    }
                    const int cls = kind == SKETCH_BF16                                      ? PSVD_KC_FUSED_BF16
                                    : (kind == SPLIT64 || kind == FINAL_SPLIT)                   ? PSVD_KC_SPLIT
                                    : kind == SPLIT3                                            ? PSVD_KC_SPLIT3
                                                                                                : PSVD_KC_FUSED_F32;
                    int pe = prof_begin(h, cls);
                    if (kind == SPLIT3) HIPCHK(h, launch_splitpass(3, fa, st));
                    else if (kind == SPLIT64) HIPCHK(h, launch_split64(fa, st));
                    else if (kind == SKETCH_BF16) HIPCHK(h, launch_sketch_bf16(fa, st));
                    else if (kind == FINAL_SPLIT) HIPCHK(h, launch_final_split(fa, st));
                    else HIPCHK(h, launch_fused(final_pass ? 1 : 0, fa, st));
                    prof_end(h, pe);
                    if (kept_gram) {
                        // G_Y from the kept Y, one partial per work-group of the pass
                        int pg = prof_begin(h, PSVD_KC_TN);
                        HIPCHK(h, launch_gram_kept(fa.yout, M, M, l, fa.nwg, fa.partG, st));
                        prof_end(h, pg);
                    }
                    FusedReduceArgs ra;
                    std::memset(&ra, 0, sizeof(ra));
                    ra.row_scale = dsc;
                    ra.nscale = r;
                    ra.partP = h->partP.as<float>();
                    ra.partG = h->partG.as<double>();
                    ra.nwg = fa.nwg;
                    ra.nlb = nlb;
                    ra.np = fa.np;
                    ra.n = n;
                    ra.lx = l;
                    ra.want_g = final_pass ? 1 : 0;
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
                if (final_pass) rc2 = tn_product(h, Y, Y, true, true, L.G_Y, nullptr, 0, nullptr, 0);
                return rc2;
            };
            for (int it = 0; it < h->q; ++it) {
                rc = pass(false);
                if (rc) return rc;
                rc = small_orth(h, L, n, l, L.X, dstat);   // X' = D orth(P)
                if (rc) return rc;
            }
            rc = pass(true);
            if (rc) return rc;
            // R_Y, Cholesky-QR2 of P, the small SVD and M2 in one work-group.
            RandFinalArgs rf;
            std::memset(&rf, 0, sizeof(rf));
            rf.n = n;
            rf.l = l;
            rf.K = h->K;
            rf.max_sweeps = h->opt.max_sweeps;
            // FP32 / mixed results carry FP32 rounding: the small SVD stops once a sweep's
            // cosines are below 2^-15 (the next sweep would leave ~2^-30); FP64 runs to m 2^-53
            rf.stop_cos2 = fp64 ? 0.0 : 0x1p-30;
            // the R factor of P = C^T Y: Cholesky-QR2; one pass with BF16 power passes,
            // whose sketch error dominates (the one-pass factor is off by about
            // kappa(P)^2 2^-53, ~1e-6 on the smallest retained value of the c2 workload)
            rf.qr_passes = prec == PSVD_PREC_BF16 ? 1 : 2;
            rf.P = L.P;
            rf.P1 = L.P1;
            rf.GY = L.G_Y;
            rf.RY = L.RY;
            rf.RYi = L.RYi;
            rf.G1 = L.H;
            rf.R1 = L.R1b;
            rf.W = L.H2;
            rf.V = L.Z;
            rf.vec = L.vec;
            rf.M2 = L.M2;
            rf.s_out = s_new;
            rf.small_u = L.sm_u;
            rf.status = dstat;
            rf.sweeps = dsweeps;
            {
                int pes = prof_begin(h, PSVD_KC_SMALL_SVD);
                HIPCHK(h, launch_small_rand_final(rf, st));
                prof_end(h, pes);
            }
            // Lift from the kept sketch: U_new = Y M2 with Y = C X (= Q R_Y).
            PanelSeg Ys = make_seg(M);
            seg_add(Ys, make_block(h->tall.p, M, tall_dtype, l));
            Ys.out = h->U[nxt].p;
            Ys.ldo = h->ldu;
            Ys.out_dtype = h->u_dtype;
            rc = lift_product(h, Ys, L.M2, l, rk, fp64, nullptr, 0, 0);
            if (rc) return rc;
            return PSVD_OK;
        };
        const bool graph = h->cstream && h->gstream && !profiling(h) && (h->opt.flags & PSVD_OPT_GRAPH);
        if (!graph) {
            rc = enqueue();
            if (rc) return rc;
        } else {
            // captured on the library's own stream (the caller's may be the null
            // stream, which cannot capture), launched on the caller's
            hipStream_t user = st;
            HIPCHK(h, hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
            st = h->stream = h->gstream;
            rc = enqueue();
            st = h->stream = user;
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(h->gstream, &g);
            if (rc || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return rc ? rc : hip_fail(h, e, "update capture");
            }
            if (h->rgraph) {
                hipGraphNode_t bad = nullptr;
                hipGraphExecUpdateResult res = hipGraphExecUpdateError;
                if (hipGraphExecUpdate(h->rgraph, g, &bad, &res) != hipSuccess || res != hipGraphExecUpdateSuccess) {
                    (void)hipGetLastError();
                    (void)hipGraphExecDestroy(h->rgraph);
                    h->rgraph = nullptr;
                }
            }
            if (!h->rgraph) e = hipGraphInstantiate(&h->rgraph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                h->rgraph = nullptr;
                return hip_fail(h, e, "update graph");
            }
            HIPCHK(h, hipGraphLaunch(h->rgraph, st));
        }
        // the test-matrix buffer is free for the upload two batches on
        if (h->cstream) HIPCHK(h, hipEventRecord(h->omega_used[ob], st));
    }
    if (h->ev1) HIPCHK(h, hipEventRecord(h->ev1, st));
    const int prev_r = h->r;
    const int64_t prev_batch = h->batch;
    h->cur = nxt;
    h->r = rk;
    h->batch += 1;
    h->stats.batches += 1;
    h->stats.last_path = randomized ? 1 : 0;
    if (h->opt.flags & PSVD_OPT_ASYNC) HIPCHK(h, launch_status_fold(dstat, st));
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
        if (h->ev0 && hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) h->stats.last_update_ms = ms;
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
    if (int rc = sync_async(h)) return rc;
    if (h->r == 0) return PSVD_OK;
    if (!out || cap < h->r) return fail(h, PSVD_E_INVAL, "output capacity below the rank");
    HIPCHK(h, hipMemcpyAsync(out, h->s[h->cur].p, (size_t)h->r * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return PSVD_OK;
}

int psvd_modes_ptr(const psvd_handle* h, const void** U, int64_t* ldu, int32_t* dtype) {
    if (!h || !U) return PSVD_E_INVAL;
    if (!h->parts.empty()) return PSVD_E_STATE;   // partitioned: psvd_pstream_modes_ptr
    *U = h->U[h->cur].p;
    if (ldu) *ldu = h->ldu;
    if (dtype) *dtype = h->u_dtype;
    return PSVD_OK;
}

int psvd_modes(const psvd_handle* hc, void* U, int64_t ldu, int32_t dtype) {
    psvd_handle* h = const_cast<psvd_handle*>(hc);
    if (!h || (!U && h->r > 0)) return PSVD_E_INVAL;
    if (!h->parts.empty()) return fail(h, PSVD_E_STATE, "partitioned handle: use psvd_pstream_modes_ptr");
    if (ldu < h->M) return fail(h, PSVD_E_SHAPE, "ldu < M");
    if (dtype != PSVD_F32 && dtype != PSVD_F64) return fail(h, PSVD_E_DTYPE, "unknown dtype");
    if (int rc = sync_async(h)) return rc;
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


// ----------------------------------------------------------------------------
// One-shot randomized SVD and checkpoints of the streaming state.
// ----------------------------------------------------------------------------
namespace {

// V[i, j] = VS[i, j] / s[j] (0 where s[j] == 0), converted to the output type.
__global__ void k_div_cols(const double* VS, int64_t n, int r, const double* s, void* V, int64_t ldv, int32_t dt) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * r) return;
    const int64_t i = e % n;
    const int j = (int)(e / n);
    const double v = s[j] > 0.0 ? VS[e] / s[j] : 0.0;
    if (dt == PSVD_F64) ((double*)V)[i + (size_t)j * ldv] = v;
    else ((float*)V)[i + (size_t)j * ldv] = (float)v;
}

int call_fail(int code, const char* msg);
}  // namespace

int psvd::set_call_error(int code, const char* msg) { return call_fail(code, msg); }

void psvd::host_omega(uint64_t seed, int64_t batch, int64_t n, int64_t l, int rounding, double* out) {
    gen_omega(seed, batch, n, l, rounding, out);
}

namespace {
int call_fail(int code, const char* msg) {
    g_call_err = std::string(status_name(code)) + ": " + msg;
    return code;
}

int rsvd_check(const void* A, int64_t M, int64_t N, int64_t lda, int32_t K, int32_t oversampling, int32_t power_iters,
               const void* U, int64_t ldu, const void* V, int64_t ldv, int32_t out_dtype) {
    if (!A || M < 1 || N < 1 || K < 1 || K > std::min<int64_t>(M, N) || oversampling < 0 || power_iters < 0)
        return call_fail(PSVD_E_INVAL, "invalid sizes or null data");
    if (lda < M || (U && ldu < M) || (V && ldv < N)) return call_fail(PSVD_E_SHAPE, "leading dimension too small");
    if (out_dtype != PSVD_F32 && out_dtype != PSVD_F64) return call_fail(PSVD_E_DTYPE, "unknown output dtype");
    return PSVD_OK;
}

// Partial-sum blocks (64 x 64 FP64 each) that tn_product writes for a
// reduction over `rows` rows into `nob` output blocks.
size_t tn_part_bytes(int64_t rows, int nob) {
    size_t most = 0;
    for (bool wide : {false, true}) {
        const int64_t chunk = tn_chunk(rows, nob, wide, 1024);
        const int64_t nitems = (rows + chunk - 1) / chunk;
        most = std::max(most, (size_t)nitems * nob * 64 * 64 * sizeof(double));
    }
    return most;
}

// The one-shot randomized SVD on a handle made for it (Eqs. 7-11): one update
// of the empty stream, then the modes (copied unless u_in_place: the update
// lifted straight into the caller's U), V = A^T U diag(1 / s) through the
// device buffer vs, and the singular values.
int rsvd_body(psvd_handle* h, const void* A, int64_t M, int64_t N, int64_t lda, int32_t a_dtype, void* U, int64_t ldu,
              bool u_in_place, void* V, int64_t ldv, int32_t out_dtype, double* s, int32_t* rank, DevBuf& vs) {
    int rc = psvd_incorporate_data(h, A, M, N, lda, a_dtype);
    if (rc) return rc;
    const int r = h->r;
    if (rank) *rank = r;
    if (U && !u_in_place) {
        rc = psvd_modes(h, U, ldu, out_dtype);
        if (rc) return rc;
    }
    if (V) {
        // V_K = A^T U_K diag(1 / s): the right factor of Eqs. (9)-(11), since
        // A^T Q U~ = B^T U~ = V~ S for B = Q^T A.
        PanelSeg L = make_seg(M);
        seg_add(L, make_block(A, lda, a_dtype, (int)N));
        PanelSeg R = make_seg(M);
        seg_add(R, make_block(h->U[h->cur].p, h->ldu, h->u_dtype, r));
        if (vs.ensure((size_t)N * r * sizeof(double)) != hipSuccess) return fail(h, PSVD_E_NOMEM, "V workspace");
        if (h->part.ensure(tn_part_bytes(M, ceil_div((int)N, 64) * ceil_div(r, 64))) != hipSuccess)
            return fail(h, PSVD_E_NOMEM, "partials");
        rc = tn_product(h, L, R, false, h->opt.precision == PSVD_PREC_FP64, vs.as<double>(), nullptr, 0, nullptr, 0);
        if (rc) return rc;
        const int64_t tot = N * r;
        hipLaunchKernelGGL(k_div_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, h->stream, vs.as<double>(), N,
                           r, h->s[h->cur].as<double>(), V, ldv, out_dtype);
        HIPCHK(h, hipGetLastError());
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    if (s) {
        rc = psvd_singular_values(h, s, h->K, nullptr);
        if (rc) return rc;
    }
    return PSVD_OK;
}

constexpr char kStateMagic[8] = {'P', 'S', 'V', 'D', 'S', 'T', '0', '1'};

struct StateHeader {
    char magic[8];
    int64_t M;
    int32_t K, r;
    double ff;
    int32_t p, q, ell, u_dtype;
    int64_t batch;
    int32_t method, precision;
    uint64_t seed;
    int64_t payload;   // bytes after the header: K doubles (s) + r columns of M (U)
};

}  // namespace

extern "C" {

int psvd_rsvd(const void* A, int64_t M, int64_t N, int64_t lda, int32_t a_dtype, int32_t K, int32_t oversampling,
              int32_t power_iters, uint64_t seed, int32_t precision, void* U, int64_t ldu, void* V, int64_t ldv,
              int32_t out_dtype, double* s, int32_t* rank, void* stream) {
    g_call_err.clear();
    if (int rc = rsvd_check(A, M, N, lda, K, oversampling, power_iters, U, ldu, V, ldv, out_dtype)) return rc;
    psvd_options o;
    psvd_default_options(&o);
    o.method = PSVD_RANDOMIZED;
    o.precision = precision;
    o.seed = seed;
    o.stream = stream;
    psvd_handle* h = nullptr;
    int rc = psvd_initialize(&h, M, K, 1.0, oversampling, power_iters, &o);
    if (rc) return call_fail(rc, "initialisation failed");
    DevBuf vs;
    rc = rsvd_body(h, A, M, N, lda, a_dtype, U, ldu, false, V, ldv, out_dtype, s, rank, vs);
    if (rc) g_call_err = h->err;
    vs.release();
    psvd_finalize(h);
    return rc;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// The one-shot randomized SVD on fixed buffers: every piece of device memory
// the update needs (partial sums, small matrices, the kept sketch, the test
// matrix, the status word, V's workspace and, when the caller passes no U, the
// modes) is carved from one caller-given device region, and the host side uses
// fixed host buffers; nothing is allocated.  The update lifts the modes straight
// into the caller's U (its element type must be the state's).
// ----------------------------------------------------------------------------
namespace psvd {

int rsvd_fixed(const FixedBuffers& fb, const void* A, int64_t M, int64_t N, int64_t lda, int32_t a_dtype, int32_t K,
               int32_t oversampling, int32_t power_iters, uint64_t seed, int32_t precision, void* U, int64_t ldu,
               void* V, int64_t ldv, int32_t out_dtype, double* s, int32_t* rank, void* stream) {
    g_call_err.clear();
    if (int rc = rsvd_check(A, M, N, lda, K, oversampling, power_iters, U, ldu, V, ldv, out_dtype)) return rc;
    if (precision < PSVD_PREC_FP64 || precision > PSVD_PREC_BF16) return call_fail(PSVD_E_INVAL, "unknown precision");
    const int32_t u_dtype = precision == PSVD_PREC_FP64 ? PSVD_F64 : PSVD_F32;
    if (a_dtype != PSVD_F32 && a_dtype != PSVD_F64) return call_fail(PSVD_E_DTYPE, "unknown dtype");
    if (a_dtype == PSVD_F64 && u_dtype != PSVD_F64) return call_fail(PSVD_E_DTYPE, "FP64 data needs FP64 precision");
    if (U && out_dtype != u_dtype)
        return call_fail(PSVD_E_DTYPE, "the allocation-free call writes U in the precision's element type");
    if (N > (1 << 20)) return call_fail(PSVD_E_SHAPE, "batch too wide");
    const int esz = u_dtype == PSVD_F64 ? 8 : 4;
    const int n = (int)N;
    const int ell = K + oversampling;
    const bool randomized = ell < n;
    const int l = randomized ? ell : 0;
    const int r = randomized ? std::min(K, l) : std::min(K, n);
    const int w = std::max(n, ell);

    // Sizes exactly as the update requests them (ensure_workspace and the
    // tall temporary), the V workspace and, without a caller U, the modes.
    size_t part = tn_part_bytes(M, ceil_div(w, 64) * (ceil_div(w, 64) + 1) / 2);
    part = std::max(part, tn_part_bytes(M, ceil_div(n, 64) * ceil_div(std::max(l, 1), 64)));
    if (V) part = std::max(part, tn_part_bytes(M, ceil_div(n, 64) * ceil_div(r, 64)));
    int np = ((n + 63) / 64) * 64;
    FusedPlan sp;
    for (int tr : {0, 32})
        if (sketch_plan(n, tr, &sp)) np = std::max(np, sp.np);
    if (fused_plan(n, 0, &sp)) np = std::max(np, sp.np);
    if (split_plan(n, &sp)) np = std::max(np, sp.np);
    const size_t wgs = std::min<size_t>(256, FU_MAX_WG);   // work-groups of a fused pass (one per CU)
    const size_t nlb = (size_t)ceil_div(std::max(ell, 1), 64);
    const int64_t ldu_state = U ? ldu : ((M + 63) / 64) * 64;
    const size_t need[] = {
        small_layout(nullptr, n, ell, K).total * sizeof(double),   // 0 small matrices
        (size_t)(3 * w + 64) * sizeof(int32_t),                     // 1 int scratch
        part,                                                       // 2 k_tn partials
        wgs * nlb * np * 64 * sizeof(float),                        // 3 fused partials
        wgs * 64 * 64 * sizeof(double),                             // 4 fused G partials
        (size_t)M * (randomized ? ell : n) * esz,                   // 5 tall temporary
        (size_t)n * std::max(ell, 1) * sizeof(double),              // 6 test matrix
        3 * (size_t)K * sizeof(double),                             // 7 s (two) and d
        64,                                                         // 8 status
        V ? (size_t)n * r * sizeof(double) : 0,                     // 9 V workspace
        U ? 0 : (size_t)ldu_state * K * esz,                        // 10 modes
    };
    constexpr int NB = (int)(sizeof(need) / sizeof(need[0]));
    size_t off[NB], total = 0;
    for (int i = 0; i < NB; ++i) {
        off[i] = total;
        total += (need[i] + 255) & ~(size_t)255;
    }
    if (total > fb.dev_bytes) {
        char msg[160];
        std::snprintf(msg, sizeof(msg), "needs %zu bytes of device scratch, the fixed maximum is %zu", total,
                      fb.dev_bytes);
        return call_fail(PSVD_E_NOMEM, msg);
    }
    if ((size_t)n * std::max(ell, 1) > fb.omega_host_entries)
        return call_fail(PSVD_E_NOMEM, "test matrix larger than the fixed host buffer");

    unsigned char* base = (unsigned char*)fb.dev;
    auto region = [&](int i) { return (void*)(base + off[i]); };
    psvd_handle hs;   // on the stack: no host allocation either
    psvd_handle* h = &hs;
    h->M = M;
    h->K = K;
    h->ff = 1.0;
    h->p = oversampling;
    h->q = power_iters;
    h->ell = ell;
    psvd_default_options(&h->opt);
    h->opt.method = PSVD_RANDOMIZED;
    h->opt.precision = precision;
    h->opt.seed = seed;
    h->opt.stream = stream;
    h->stream = (hipStream_t)stream;
    h->u_dtype = u_dtype;
    h->ldu = ldu_state;
    std::memset(&h->stats, 0, sizeof(h->stats));
    if (hipGetDevice(&h->device) != hipSuccess) return call_fail(PSVD_E_DEVICE, "hipGetDevice");
    void* ubuf = U ? U : region(10);
    h->U[0].borrow(ubuf, (size_t)ldu_state * K * esz);   // r = 0: the update reads no previous modes
    h->U[1].borrow(ubuf, (size_t)ldu_state * K * esz);
    double* sd = (double*)region(7);
    h->s[0].borrow(sd, K * sizeof(double));
    h->s[1].borrow(sd + K, K * sizeof(double));
    h->d.borrow(sd + 2 * K, K * sizeof(double));
    h->small.borrow(region(0), need[0]);
    h->ivec.borrow(region(1), need[1]);
    h->part.borrow(region(2), need[2]);
    h->partP.borrow(region(3), need[3]);
    h->partG.borrow(region(4), need[4]);
    h->tall.borrow(region(5), need[5]);
    h->omega_dev[0].borrow(region(6), need[6]);
    h->status.borrow(region(8), need[8]);
    h->status_host = fb.status_host;
    h->omega_host[0] = fb.omega_host;
    h->omega_host_cap = fb.omega_host_entries;
    h->nmax = n;   // the workspace above is sized for this panel
    DevBuf vs;
    vs.borrow(region(9), need[9]);
    // The region keeps the previous call's contents.  Nothing needs clearing
    // here: the update's first kernel zeroes the status words, the previous
    // singular values are read only for r > 0 columns (none), and every partial
    // sum, small matrix and tall temporary is written before it is read.
    int rc = rsvd_body(h, A, M, N, lda, a_dtype, U, ldu, true, V, ldv, out_dtype, s, rank, vs);
    if (rc) g_call_err = h->err;
    (void)hipStreamSynchronize(h->stream);
    return rc;
}

}  // namespace psvd

extern "C" {

int psvd_save_state(const psvd_handle* hc, void* buf, size_t cap, size_t* size) {
    psvd_handle* h = const_cast<psvd_handle*>(hc);
    if (!h) return PSVD_E_INVAL;
    if (!h->parts.empty()) return fail(h, PSVD_E_STATE, "checkpoints cover single-panel handles");
    const int esz = h->u_dtype == PSVD_F64 ? 8 : 4;
    const size_t payload = (size_t)h->K * sizeof(double) + (size_t)h->r * h->M * esz;
    const size_t total = sizeof(StateHeader) + payload;
    if (size) *size = total;
    if (!buf) return PSVD_OK;
    if (int rc = sync_async(h)) return rc;
    if (cap < total) return fail(h, PSVD_E_INVAL, "buffer smaller than the state");
    StateHeader hd;
    std::memset(&hd, 0, sizeof(hd));
    std::memcpy(hd.magic, kStateMagic, 8);
    hd.M = h->M;
    hd.K = h->K;
    hd.r = h->r;
    hd.ff = h->ff;
    hd.p = h->p;
    hd.q = h->q;
    hd.ell = h->ell;
    hd.u_dtype = h->u_dtype;
    hd.batch = h->batch;
    hd.method = h->opt.method;
    hd.precision = h->opt.precision;
    hd.seed = h->opt.seed;
    hd.payload = (int64_t)payload;
    char* out = (char*)buf;
    std::memcpy(out, &hd, sizeof(hd));
    double* sv = (double*)(out + sizeof(hd));
    std::memset(sv, 0, (size_t)h->K * sizeof(double));
    if (h->r > 0) {
        HIPCHK(h, hipMemcpyAsync(sv, h->s[h->cur].p, (size_t)h->r * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipMemcpy2DAsync(out + sizeof(hd) + (size_t)h->K * sizeof(double), (size_t)h->M * esz, h->U[h->cur].p,
                                   (size_t)h->ldu * esz, (size_t)h->M * esz, h->r, hipMemcpyDeviceToHost, h->stream));
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return PSVD_OK;
}

int psvd_load_state(psvd_handle* h, const void* buf, size_t size) {
    if (!h || !buf) return PSVD_E_INVAL;
    h->err.clear();
    if (!h->parts.empty()) return fail(h, PSVD_E_STATE, "checkpoints cover single-panel handles");
    StateHeader hd;
    if (size < sizeof(hd)) return fail(h, PSVD_E_INVAL, "buffer shorter than the state header");
    std::memcpy(&hd, buf, sizeof(hd));
    if (std::memcmp(hd.magic, kStateMagic, 8) != 0) return fail(h, PSVD_E_INVAL, "not a state buffer");
    if (hd.M != h->M || hd.K != h->K || hd.ff != h->ff || hd.p != h->p || hd.q != h->q || hd.ell != h->ell ||
        hd.u_dtype != h->u_dtype || hd.method != h->opt.method || hd.precision != h->opt.precision ||
        hd.seed != h->opt.seed)
        return fail(h, PSVD_E_STATE, "state saved with a different configuration");
    const int esz = h->u_dtype == PSVD_F64 ? 8 : 4;
    if (hd.r < 0 || hd.r > h->K || hd.batch < 0) return fail(h, PSVD_E_INVAL, "corrupt state header");
    const size_t payload = (size_t)h->K * sizeof(double) + (size_t)hd.r * h->M * esz;
    if ((size_t)hd.payload != payload || size < sizeof(hd) + payload) return fail(h, PSVD_E_INVAL, "truncated state");
    const char* in = (const char*)buf + sizeof(hd);
    // write into the idle buffer pair, then make it current (the state changes only on success)
    const int nxt = 1 - h->cur;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (hd.r > 0) {
        HIPCHK(h, hipMemcpyAsync(h->s[nxt].p, in, (size_t)hd.r * sizeof(double), hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpy2DAsync(h->U[nxt].p, (size_t)h->ldu * esz, in + (size_t)h->K * sizeof(double),
                                   (size_t)h->M * esz, (size_t)h->M * esz, hd.r, hipMemcpyHostToDevice, h->stream));
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->cur = nxt;
    h->r = hd.r;
    h->batch = hd.batch;
    return PSVD_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// Reverse mode of the deterministic stream.
// ----------------------------------------------------------------------------
namespace {

struct GradCtx {
    psvd_handle* h = nullptr;       // deterministic handle that runs the forward
    int64_t M = 0;
    int B = 0;
    int64_t Nb = 0;
    int K = 0;
    int dt = PSVD_F32;
    int esz = 4;
    DevBuf Ust, sst;                // states entering every batch
    std::vector<int> rst;
    DevBuf Ubar[2];                 // cotangent of the current U (M x K)
    DevBuf work;                    // small FP64 matrices
    ~GradCtx() {
        if (h) psvd_finalize(h);
    }
};

// Forward pass storing the state that enters every batch.
int grad_forward(GradCtx& g, const void* A, int64_t lda, double ff, hipStream_t st, bool store) {
    psvd_options o;
    psvd_default_options(&o);
    o.method = PSVD_DETERMINISTIC;
    o.precision = g.dt == PSVD_F64 ? PSVD_PREC_FP64 : PSVD_PREC_FP32;
    o.stream = st;
    o.flags = PSVD_OPT_NO_FALLBACK;
    int rc = psvd_initialize(&g.h, g.M, g.K, ff, 0, 0, &o);
    if (rc) return rc;
    psvd_handle* h = g.h;
    if (store) {
        HIPCHK(h, g.Ust.ensure((size_t)g.B * h->ldu * g.K * g.esz));
        HIPCHK(h, g.sst.ensure((size_t)g.B * g.K * sizeof(double)));
        g.rst.assign(g.B, 0);
    }
    for (int b = 0; b < g.B; ++b) {
        if (store) {
            g.rst[b] = h->r;
            HIPCHK(h, hipMemcpyAsync((char*)g.Ust.p + (size_t)b * h->ldu * g.K * g.esz, h->U[h->cur].p,
                                     (size_t)h->ldu * g.K * g.esz, hipMemcpyDeviceToDevice, st));
            HIPCHK(h, hipMemcpyAsync(g.sst.as<double>() + (size_t)b * g.K, h->s[h->cur].p, g.K * sizeof(double),
                                     hipMemcpyDeviceToDevice, st));
        }
        const void* Ab = (const char*)A + (size_t)b * g.Nb * lda * g.esz;
        rc = psvd_incorporate_data(h, Ab, g.M, g.Nb, lda, g.dt);
        if (rc) return rc;
    }
    return PSVD_OK;
}

// Carry (U_bar, s_bar) of the final state back through every batch; the data
// part of each panel cotangent is written (or added, accumulate) to A_bar.
int grad_backward(GradCtx& g, const void* A, int64_t lda, double ff, const double* sbar_host, void* Abar,
                  int accumulate, hipStream_t st) {
    psvd_handle* h = g.h;
    const int K = g.K;
    const int nmax = K + (int)g.Nb;
    int rc = ensure_workspace(h, nmax);
    if (rc) return rc;
    HIPCHK(h, h->tall.ensure((size_t)g.M * nmax * g.esz));
    // work layout
    size_t nn = (size_t)nmax * nmax, nk = (size_t)nmax * K, zz = (size_t)(nmax + K) * nmax;
    const size_t words = 8 * nn + 2 * nk + 2 * zz + (size_t)K * K + 4 * (size_t)nmax + 256;
    HIPCHK(h, g.work.ensure(words * sizeof(double)));
    double* w = g.work.as<double>();
    double *gR = w, *gUt = gR + nn, *gT = gUt + nn, *gTf = gT + nn, *gV = gTf + nn, *gWk = gV + nn, *gZt = gWk + nn;
    double *gE = gZt + nn, *gH = gE + nk, *gZu = gH + nk, *gZa = gZu + zz, *gGrr = gZa + zz;
    double *gS = gGrr + (size_t)K * K, *gsbar = gS + nmax, *gd = gsbar + nmax;
    int32_t* dstat = h->status.as<int32_t>();
    const bool fp64 = g.dt == PSVD_F64;
    int r_fin = h->r;
    HIPCHK(h, hipMemsetAsync(gsbar, 0, sizeof(double) * nmax, st));
    HIPCHK(h, hipMemcpyAsync(gsbar, sbar_host, sizeof(double) * r_fin, hipMemcpyHostToDevice, st));
    int cb = 0;   // Ubar[cb] holds the current cotangent
    for (int b = g.B - 1; b >= 0; --b) {
        const int r = g.rst[b];
        const int n = r + (int)g.Nb;
        const int rk = std::min(K, n);
        const void* Ub = (const char*)g.Ust.p + (size_t)b * h->ldu * K * g.esz;
        const double* sb = g.sst.as<double>() + (size_t)b * K;
        const void* Ab = (const char*)A + (size_t)b * g.Nb * lda * g.esz;
        HIPCHK(h, launch_make_scale(dstat, gd, sb, r, ff, st));
        PanelSeg C = make_seg(g.M);
        if (r > 0) seg_add(C, make_block(Ub, h->ldu, g.dt, r));
        seg_add(C, make_block(Ab, lda, g.dt, (int)g.Nb));
        SmallLayout L = small_layout(h->small.as<double>(), n, 0, K);
        // Recompute the full thin SVD of the panel: Cholesky-QR2 + Jacobi of R.
        rc = tn_product(h, C, C, true, true, L.G, nullptr, 0, nullptr, 0);
        if (rc) return rc;
        SmallArgs sa;
        std::memset(&sa, 0, sizeof(sa));
        sa.n = n;
        sa.r = r;
        sa.K = n;                 // keep every triplet
        sa.max_sweeps = h->opt.max_sweeps;
        sa.allow_fallback = 0;
        sa.d = gd;
        sa.G = gR;                // det1 scales G here; det2 leaves R = R2 R1 here
        sa.G2 = L.G2;
        sa.R1 = L.R1;
        sa.Ri = L.Ri;
        sa.Z = L.Z;
        sa.T = gT;
        sa.Xn = L.Xn;
        sa.s_out = gS;
        sa.small_u = gUt;
        sa.vec = L.vec;
        sa.ivec = h->ivec.as<int32_t>();
        sa.status = dstat;
        sa.sweeps = dstat + 1;
        HIPCHK(h, hipMemcpyAsync(gR, L.G, sizeof(double) * n * n, hipMemcpyDeviceToDevice, st));
        {
            int pes = prof_begin(h, PSVD_KC_SMALL_SVD);
            HIPCHK(h, launch_small_det1(sa, st));
            prof_end(h, pes);
        }
        PanelSeg Q = C;
        Q.out = h->tall.p;
        Q.ldo = g.M;
        Q.out_dtype = h->u_dtype;
        rc = nn_product(h, Q, L.Xn, n, n, fp64, nullptr, 0, dstat, DEV_NONFINITE | DEV_BREAKDOWN);
        if (rc) return rc;
        PanelSeg Q1 = make_seg(g.M);
        seg_add(Q1, make_block(h->tall.p, g.M, h->u_dtype, n));
        rc = tn_product(h, Q1, Q1, true, true, L.G2, nullptr, 0, dstat, DEV_NONFINITE | DEV_BREAKDOWN);
        if (rc) return rc;
        {
            int pes = prof_begin(h, PSVD_KC_SMALL_SVD);
            HIPCHK(h, launch_small_det2(sa, st));
            prof_end(h, pes);
        }
        // E = C^T U_bar (C with its column scale).
        PanelSeg Ubs = make_seg(g.M);
        seg_add(Ubs, make_block(g.Ubar[cb].p, g.M, g.dt, rk));
        rc = tn_product(h, C, Ubs, false, true, gE, gd, r, nullptr, 0);
        if (rc) return rc;
        GradCoreArgs ga;
        ga.n = n;
        ga.r = r;
        ga.rk = rk;
        ga.R = gR;
        ga.Ut = gUt;
        ga.S = gS;
        ga.E = gE;
        ga.sbar = gsbar;
        ga.d = gd;
        ga.Tf = gTf;
        ga.V = gV;
        ga.H = gH;
        ga.Wk = gWk;
        ga.Zt = gZt;
        ga.Zu = gZu;
        ga.Za = gZa;
        ga.status = dstat;
        HIPCHK(h, launch_grad_core(ga, st));
        // C_bar = [U_prev | A_b | U_bar] [Z]: data part -> A_bar, U part -> next cotangent.
        PanelSeg P3 = C;
        seg_add(P3, make_block(g.Ubar[cb].p, g.M, g.dt, rk));
        P3.out = (char*)Abar + (size_t)b * g.Nb * g.M * g.esz;
        P3.ldo = g.M;
        P3.out_dtype = g.dt;
        rc = nn_product(h, P3, gZa, n + rk, (int)g.Nb, fp64, nullptr, 0, dstat, DEV_NONFINITE | DEV_BREAKDOWN | DEV_NOCONV,
                        PSVD_KC_LIFT, 0, accumulate);
        if (rc) return rc;
        if (r > 0) {
            PanelSeg P3u = P3;
            P3u.out = g.Ubar[1 - cb].p;
            rc = nn_product(h, P3u, gZu, n + rk, r, fp64, nullptr, 0, dstat, DEV_NONFINITE | DEV_BREAKDOWN | DEV_NOCONV,
                            PSVD_KC_LIFT);
            if (rc) return rc;
            PanelSeg Us = make_seg(g.M);
            seg_add(Us, make_block(Ub, h->ldu, g.dt, r));
            PanelSeg Un = make_seg(g.M);
            seg_add(Un, make_block(g.Ubar[1 - cb].p, g.M, g.dt, r));
            rc = tn_product(h, Us, Un, false, true, gGrr, nullptr, 0, nullptr, 0);
            if (rc) return rc;
            HIPCHK(h, hipMemsetAsync(gsbar, 0, sizeof(double) * nmax, st));
            HIPCHK(h, launch_grad_sbar(gGrr, r, sb, gsbar, st));
            cb = 1 - cb;
        }
        int32_t hs[2] = {0, 0};
        HIPCHK(h, hipMemcpyAsync(hs, dstat, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(h, hipStreamSynchronize(st));
        if (hs[0] & (DEV_BREAKDOWN | DEV_FALLBACK))
            return fail(h, PSVD_E_BREAKDOWN, "rank-deficient panel: the adjoint needs a full-rank batch");
        int code = finish_status(h, hs[0]);
        if (code) return code;
    }
    return PSVD_OK;
}

int grad_setup(GradCtx& g, const void* A, int64_t M, int64_t lda, int32_t dtype, int32_t B, int64_t Nb, int32_t K) {
    if (!A || M < 1 || B < 1 || Nb < 1 || K < 1 || K > M || lda < M) return PSVD_E_INVAL;
    if (dtype != PSVD_F32 && dtype != PSVD_F64) return PSVD_E_DTYPE;
    if ((int64_t)K + Nb > M) return PSVD_E_SHAPE;
    g.M = M;
    g.B = B;
    g.Nb = Nb;
    g.K = K;
    g.dt = dtype;
    g.esz = dtype == PSVD_F64 ? 8 : 4;
    return PSVD_OK;
}

}  // namespace

extern "C" int psvd_stream_backward(const void* A, int64_t M, int64_t lda, int32_t dtype, int32_t B, int64_t Nb,
                                    int32_t K, double ff, const void* U_bar, const double* s_bar, void* A_bar,
                                    void* stream) {
    GradCtx g;
    int rc = grad_setup(g, A, M, lda, dtype, B, Nb, K);
    if (rc) return rc;
    if (!U_bar || !s_bar || !A_bar || !(ff > 0.0 && ff <= 1.0)) return PSVD_E_INVAL;
    hipStream_t st = (hipStream_t)stream;
    rc = grad_forward(g, A, lda, ff, st, true);
    if (rc) return rc;
    psvd_handle* h = g.h;
    const int r = h->r;
    for (int b = 0; b < 2; ++b) HIPCHK(h, g.Ubar[b].ensure((size_t)M * K * g.esz));
    HIPCHK(h, hipMemsetAsync(g.Ubar[0].p, 0, (size_t)M * K * g.esz, st));
    HIPCHK(h, hipMemcpyAsync(g.Ubar[0].p, U_bar, (size_t)M * r * g.esz, hipMemcpyDeviceToDevice, st));
    rc = grad_backward(g, A, lda, ff, s_bar, A_bar, 0, st);
    if (rc) return rc;
    HIPCHK(h, hipStreamSynchronize(st));
    return PSVD_OK;
}

extern "C" int psvd_loss_grad(const void* A, int64_t M, int64_t lda, int32_t dtype, int32_t B, int64_t Nb,
                              int32_t K, double ff, const double* w, double* loss, void* grad, void* stream) {
    GradCtx g;
    int rc = grad_setup(g, A, M, lda, dtype, B, Nb, K);
    if (rc) return rc;
    if (!w || !(ff > 0.0 && ff <= 1.0)) return PSVD_E_INVAL;
    hipStream_t st = (hipStream_t)stream;
    rc = grad_forward(g, A, lda, ff, st, grad != nullptr);
    if (rc) return rc;
    psvd_handle* h = g.h;
    const int r = h->r;
    const int Nt = B * (int)Nb;
    // W = U^T A (r x Nt) and the column norms of A, both in FP64.
    PanelSeg Us = make_seg(M);
    seg_add(Us, make_block(h->U[h->cur].p, h->ldu, g.dt, r));
    PanelSeg As = make_seg(M);
    seg_add(As, make_block(A, lda, dtype, Nt));
    DevBuf tmp;
    HIPCHK(h, tmp.ensure(sizeof(double) * ((size_t)r * Nt + (size_t)Nt * Nt + (size_t)(Nt + r) * Nt + 64)));
    double* dW = tmp.as<double>();
    double* dAA = dW + (size_t)r * Nt;
    double* dX = dAA + (size_t)Nt * Nt;
    rc = tn_product(h, Us, As, false, true, dW, nullptr, 0, nullptr, 0);
    if (rc) return rc;
    rc = tn_product(h, As, As, true, true, dAA, nullptr, 0, nullptr, 0);
    if (rc) return rc;
    std::vector<double> W((size_t)r * Nt), AA((size_t)Nt * Nt), s(r);
    HIPCHK(h, hipMemcpyAsync(W.data(), dW, sizeof(double) * W.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipMemcpyAsync(AA.data(), dAA, sizeof(double) * AA.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipMemcpyAsync(s.data(), h->s[h->cur].p, sizeof(double) * r, hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
    double a2 = 0.0, p2 = 0.0, ws = 0.0;
    for (int j = 0; j < Nt; ++j) a2 += AA[(size_t)j * Nt + j];
    for (double v : W) p2 += v * v;
    for (int j = 0; j < r; ++j) ws += w[j] * s[j];
    if (loss) *loss = a2 - p2 + ws;
    if (!grad) return PSVD_OK;
    // Direct term: grad = [A | U] [2 I; -2 W].
    std::vector<double> X((size_t)(Nt + r) * Nt, 0.0);
    for (int j = 0; j < Nt; ++j) {
        X[(size_t)j * (Nt + r) + j] = 2.0;
        for (int i = 0; i < r; ++i) X[(size_t)j * (Nt + r) + Nt + i] = -2.0 * W[(size_t)j * r + i];
    }
    HIPCHK(h, hipMemcpyAsync(dX, X.data(), sizeof(double) * X.size(), hipMemcpyHostToDevice, st));
    PanelSeg AU = As;
    seg_add(AU, make_block(h->U[h->cur].p, h->ldu, g.dt, r));
    AU.out = grad;
    AU.ldo = M;
    AU.out_dtype = dtype;
    rc = nn_product(h, AU, dX, Nt + r, Nt, g.dt == PSVD_F64, nullptr, 0, nullptr, 0);
    if (rc) return rc;
    HIPCHK(h, hipStreamSynchronize(st));
    // Final cotangents: U_bar = -2 A W^T, s_bar = w.
    for (int b = 0; b < 2; ++b) HIPCHK(h, g.Ubar[b].ensure((size_t)M * K * g.esz));
    std::vector<double> Wt((size_t)Nt * r);
    for (int j = 0; j < Nt; ++j)
        for (int i = 0; i < r; ++i) Wt[(size_t)i * Nt + j] = -2.0 * W[(size_t)j * r + i];
    HIPCHK(h, hipMemcpyAsync(dX, Wt.data(), sizeof(double) * Wt.size(), hipMemcpyHostToDevice, st));
    PanelSeg Ao = As;
    Ao.out = g.Ubar[0].p;
    Ao.ldo = M;
    Ao.out_dtype = dtype;
    rc = nn_product(h, Ao, dX, Nt, r, g.dt == PSVD_F64, nullptr, 0, nullptr, 0);
    if (rc) return rc;
    HIPCHK(h, hipStreamSynchronize(st));
    rc = grad_backward(g, A, lda, ff, w, grad, 1, st);
    if (rc) return rc;
    HIPCHK(h, hipStreamSynchronize(st));
    return PSVD_OK;
}

// ----------------------------------------------------------------------------
// Partitioned streaming: the parallel streaming SVD of Section 3 with the P
// row partitions on this device.  The first batch initialises U and s with
// APMOS (Algorithm 2); each later batch combines the partitions' QR factors.
// With the Cholesky-based QR the R factor of partition i comes from its Gram
// G_i = C_i^T C_i, and the QR of the stacked R factors [R_1; ..; R_P] has
// the R factor of their Gram sum_i R_i^T R_i = sum_i G_i: the partitions'
// Gram partials are summed in one fixed-order reduction (the all-reduce of a
// distributed run), the small core is the serial one, and every partition's
// lift uses the same small factor (Q_g^i = R_i R_f^-1, so Q_i Q_g^i = C_i R_f^-1).
// ----------------------------------------------------------------------------
namespace {

// One panel per partition: [U_i | A_i] with output rows of U_new_i.
std::vector<PanelSeg> part_panels(const psvd_handle* h, int r, const void* const* A, const int64_t* ld, int32_t dt,
                                  int N, const void* Ucur, void* Unew) {
    const int esz = h->u_dtype == PSVD_F64 ? 8 : 4;
    std::vector<PanelSeg> segs(h->parts.size());
    for (size_t i = 0; i < h->parts.size(); ++i) {
        const int64_t Mi = h->parts[i];
        PanelSeg C = make_seg(Mi);
        if (r > 0) seg_add(C, make_block((const char*)Ucur + (size_t)h->poff[i] * h->K * esz, Mi, h->u_dtype, r));
        seg_add(C, make_block(A[i], ld[i], dt, N));
        C.out = (char*)Unew + (size_t)h->poff[i] * h->K * esz;
        C.ldo = Mi;
        C.out_dtype = h->u_dtype;
        segs[i] = C;
    }
    return segs;
}

}  // namespace

// Device copies of the partition panels and of their row chunks: one launch
// covers every partition (a chunk is (partition, first row, end row)).
struct PartLists {
    const PanelSeg* segs = nullptr;
    const WorkItem* items = nullptr;
    int nitems = 0;
    int64_t chunk = 0;
    bool vec = false;   // every segment takes 16-byte column loads (seg_vec_ok)
    int dtype_all = 0;  // the dtype of every column of every segment, or 0
};

static std::vector<WorkItem> part_items(const psvd_handle* h, int64_t chunk) {
    std::vector<WorkItem> it;
    for (size_t i = 0; i < h->parts.size(); ++i)
        for (int64_t r0 = 0; r0 < h->parts[i]; r0 += chunk) {
            WorkItem w;
            w.seg = (int32_t)i;
            w.pad = 0;
            w.row0 = r0;
            w.row1 = std::min<int64_t>(r0 + chunk, h->parts[i]);
            it.push_back(w);
        }
    return it;
}

// out (nl x nl FP64, symmetric) = sum_i S_i^T S_i: the partials of every
// partition's row chunks are summed in one fixed-order reduction.
static int tn_product_parts(psvd_handle* h, const PanelSeg& S0, const PartLists& pl, int nob, int mbl, bool fp64,
                            double* out, const int32_t* skip, int skip_mask) {
    HIPCHK(h, h->part.ensure((size_t)pl.nitems * nob * 64 * 64 * sizeof(double)));
    TnArgs a;
    std::memset(&a, 0, sizeof(a));
    a.lseg = S0;
    a.rseg = S0;
    a.lsegs = pl.segs;
    a.rsegs = pl.segs;
    a.items = pl.items;
    a.chunk = pl.chunk;
    a.mbl = mbl;
    a.sym = 1;
    a.part = h->part.as<double>();
    a.skip = skip;
    a.skip_mask = skip_mask;
    a.nob = nob;
    a.vec = pl.vec ? 1 : 0;
    a.dtype_all = pl.dtype_all;
    int pe = prof_begin(h, PSVD_KC_TN);
    HIPCHK(h, launch_tn(fp64, a, pl.nitems, h->stream));
    prof_end(h, pe);
    TnReduceArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.part = h->part.as<double>();
    ra.seg_item0 = nullptr;
    ra.nitems = pl.nitems;
    ra.mbl = mbl;
    ra.nob = nob;
    ra.nl = S0.ncols;
    ra.nr = S0.ncols;
    ra.sym = 1;
    ra.out = out;
    ra.skip = skip;
    ra.skip_mask = skip_mask;
    HIPCHK(h, launch_tn_reduce(ra, 1, h->stream));
    return PSVD_OK;
}

// out_i (partition panels' outputs) = S_i X for every partition in one launch.
static int nn_product_parts(psvd_handle* h, const PanelSeg& S0, const PartLists& pl, const double* X, int64_t ldx,
                            int nx, bool fp64, const int32_t* skip, int skip_mask, int cls, int need_mask = 0) {
    NnArgs a;
    std::memset(&a, 0, sizeof(a));
    a.seg = S0;
    a.segs = pl.segs;
    a.items = pl.items;
    a.chunk = pl.chunk;
    a.X = X;
    a.ldx = ldx;
    a.n = S0.ncols;
    a.nx = nx;
    a.skip = skip;
    a.skip_mask = skip_mask;
    a.need_mask = need_mask;
    a.vec16 = pl.vec ? 1 : 0;
    int pe = prof_begin(h, cls);
    HIPCHK(h, launch_nn(fp64, a, pl.nitems, h->stream));
    prof_end(h, pe);
    return PSVD_OK;
}

extern "C" {

int psvd_pstream_initialize(psvd_handle** out, int32_t P, const int64_t* M_parts, int32_t K, double ff,
                            int32_t r_local, const psvd_options* opt) {
    if (!out) return PSVD_E_INVAL;
    *out = nullptr;
    if (P < 1 || !M_parts || K < 1 || r_local < 0) return PSVD_E_INVAL;
    int64_t M = 0;
    for (int i = 0; i < P; ++i) {
        if (M_parts[i] < 1) return PSVD_E_INVAL;
        M += M_parts[i];
    }
    psvd_options o;
    psvd_default_options(&o);
    if (opt) o = *opt;
    if (o.precision == PSVD_PREC_MIXED || o.precision == PSVD_PREC_BF16) return PSVD_E_INVAL;
    // PSVD_RANDOMIZED: the paper's placement of randomization in the parallel
    // variant -- the SVD of W (initialisation) and of the combined R factor
    // (updates) by the low-rank SVD with a K-column test matrix (ell = K)
    psvd_handle* h = nullptr;
    int rc = psvd_initialize(&h, M, K, ff, 0, 0, &o);
    if (rc) return rc;
    h->parts.assign(M_parts, M_parts + P);
    h->poff.resize(P);
    int64_t off = 0;
    for (int i = 0; i < P; ++i) {
        h->poff[i] = off;
        off += M_parts[i];
    }
    h->r_local = r_local;
    *out = h;
    return PSVD_OK;
}

int psvd_pstream_incorporate(psvd_handle* h, const void* const* A_parts, const int64_t* ld_parts, int64_t N,
                             int32_t dtype) {
    if (!h) return PSVD_E_INVAL;
    h->err.clear();
    if (h->parts.empty()) return fail(h, PSVD_E_STATE, "not a partitioned handle");
    const int P = (int)h->parts.size();
    if (N < 0 || (N > 0 && (!A_parts || !ld_parts))) return fail(h, PSVD_E_INVAL, "N < 0 or null data");
    if (dtype != h->u_dtype) return fail(h, PSVD_E_DTYPE, "partition data must have the state's element type");
    if (N == 0) return PSVD_OK;
    if (N > 1 << 20) return fail(h, PSVD_E_SHAPE, "batch too wide");
    for (int i = 0; i < P; ++i) {
        if (!A_parts[i]) return fail(h, PSVD_E_INVAL, "null partition");
        if (ld_parts[i] < h->parts[i]) return fail(h, PSVD_E_SHAPE, "partition leading dimension < M_i");
    }
    if (int rc = sync_async(h)) return rc;
    const int esz = h->u_dtype == PSVD_F64 ? 8 : 4;
    hipStream_t st = h->stream;
    if (h->r == 0) {
        // ---- initialisation: APMOS over the partitions ----
        const int rl = h->r_local > 0 ? h->r_local : (int)std::min<int64_t>(h->K, N);
        if (h->K > N || rl > N) return fail(h, PSVD_E_SHAPE, "the first batch needs K <= N and r_local <= N");
        std::vector<void*> Up(P);
        std::vector<int64_t> ldu(P);
        for (int i = 0; i < P; ++i) {
            Up[i] = (char*)h->U[h->cur].p + (size_t)h->poff[i] * h->K * esz;
            ldu[i] = h->parts[i];
        }
        std::vector<double> lam(h->K);
        const int ell0 = h->ell > 0 ? h->K : 0;
        int rc = apmos_internal(P, A_parts, h->parts.data(), ld_parts, N, dtype, rl, h->K, ell0, h->opt.seed, h->batch,
                                Up.data(), ldu.data(), lam.data(), nullptr, st);
        if (rc) return fail(h, rc, std::string("APMOS initialisation: ") + psvd_status_string(rc));
        HIPCHK(h, hipMemcpyAsync(h->s[h->cur].p, lam.data(), sizeof(double) * h->K, hipMemcpyHostToDevice, st));
        HIPCHK(h, hipStreamSynchronize(st));
        h->r = h->K;
        h->batch += 1;
        h->stats.batches += 1;
        return PSVD_OK;
    }
    // ---- update: Cholesky-QR2 of the partitioned panel + Jacobi SVD of R ----
    const int r = h->r;
    const int n = r + (int)N;
    for (int i = 0; i < P; ++i)
        if (h->parts[i] < n) return fail(h, PSVD_E_SHAPE, "a partition has fewer rows than the panel has columns");
    int rc = ensure_workspace(h, n);
    if (rc) return rc;
    HIPCHK(h, h->tall.ensure((size_t)h->M * n * esz));
    const bool fp64 = h->opt.precision == PSVD_PREC_FP64;
    const int rk = std::min<int>(h->K, n);
    SmallLayout L = small_layout(h->small.as<double>(), n, 0, h->K);
    int32_t* dstat = h->status.as<int32_t>();
    const int cur = h->cur, nxt = 1 - cur;
    double* s_cur = h->s[cur].as<double>();
    double* s_new = h->s[nxt].as<double>();
    HIPCHK(h, hipEventRecord(h->ev0, st));
    HIPCHK(h, launch_make_scale(dstat, h->d.as<double>(), s_cur, r, h->ff, st));
    std::vector<PanelSeg> C = part_panels(h, r, A_parts, ld_parts, dtype, (int)N, h->U[cur].p, h->U[nxt].p);
    // Q1_i (tall temporary, partition i at rows poff[i] with leading dimension M_i)
    std::vector<PanelSeg> Q1(P), Qin(P);
    for (int i = 0; i < P; ++i) {
        char* q = (char*)h->tall.p + (size_t)h->poff[i] * n * esz;
        Qin[i] = C[i];
        Qin[i].out = q;
        Qin[i].ldo = h->parts[i];
        Qin[i].out_dtype = h->u_dtype;
        Q1[i] = make_seg(h->parts[i]);
        seg_add(Q1[i], make_block(q, h->parts[i], h->u_dtype, n));
        Q1[i].out = C[i].out;
        Q1[i].ldo = C[i].ldo;
        Q1[i].out_dtype = h->u_dtype;
    }
    // descriptors: [C panels | Q1 panels | C panels writing Q1 | Gram chunks | product chunks]
    const int mbl = ceil_div(n, 64), nob = mbl * (mbl + 1) / 2;
    bool cvec = true, qvec = true;   // 16-byte column loads for every partition
    int cdt = seg_dtype_all(C[0]), qdt = seg_dtype_all(Q1[0]);
    for (int i = 0; i < P; ++i) {
        cvec = cvec && seg_vec_ok(C[i], false);
        qvec = qvec && seg_vec_ok(Q1[i], false);
        if (seg_dtype_all(C[i]) != cdt) cdt = 0;
        if (seg_dtype_all(Q1[i]) != qdt) qdt = 0;
    }
    // one chunk for both Grams (their items share a descriptor list): the
    // whole-Gram chunk when both take k_tn_w
    const int64_t tchunk = (tn_wide(true, mbl, cdt) && tn_wide(true, mbl, qdt))
                               ? chunk_for_items(h->parts.data(), P, TN_WIDE_ITEMS)
                               : pick_chunk(h->M, nob, 64, split_items(h));
    const std::vector<WorkItem> tit = part_items(h, tchunk);
    const int64_t nchunk = pick_chunk(h->M, ceil_div(n, 64), 64, split_items(h));
    const std::vector<WorkItem> nit = part_items(h, nchunk);
    {
        const size_t bytes = sizeof(PanelSeg) * 3 * P + sizeof(WorkItem) * (tit.size() + nit.size());
        HIPCHK(h, h->pdesc.ensure(bytes));
        std::vector<unsigned char> host(bytes);
        unsigned char* q = host.data();
        std::memcpy(q, C.data(), sizeof(PanelSeg) * P);
        std::memcpy(q + sizeof(PanelSeg) * P, Q1.data(), sizeof(PanelSeg) * P);
        std::memcpy(q + sizeof(PanelSeg) * 2 * P, Qin.data(), sizeof(PanelSeg) * P);
        std::memcpy(q + sizeof(PanelSeg) * 3 * P, tit.data(), sizeof(WorkItem) * tit.size());
        std::memcpy(q + sizeof(PanelSeg) * 3 * P + sizeof(WorkItem) * tit.size(), nit.data(),
                    sizeof(WorkItem) * nit.size());
        HIPCHK(h, hipMemcpyAsync(h->pdesc.p, host.data(), bytes, hipMemcpyHostToDevice, st));
        HIPCHK(h, hipStreamSynchronize(st));   // the host staging vector goes out of scope
    }
    const PanelSeg* dC = h->pdesc.as<PanelSeg>();
    const PanelSeg* dQ = dC + P;
    const PanelSeg* dQin = dQ + P;
    const WorkItem* dT = (const WorkItem*)(dQin + P);
    const WorkItem* dN = dT + tit.size();
    PartLists cg{dC, dT, (int)tit.size(), tchunk}, qg{dQ, dT, (int)tit.size(), tchunk};
    PartLists cn{dC, dN, (int)nit.size(), nchunk}, qn{dQ, dN, (int)nit.size(), nchunk};
    PartLists qin{dQin, dN, (int)nit.size(), nchunk};
    cg.vec = cn.vec = qin.vec = cvec;
    qg.vec = qn.vec = qvec;
    cg.dtype_all = cdt;
    qg.dtype_all = qdt;
    rc = tn_product_parts(h, C[0], cg, nob, mbl, true, L.G, nullptr, 0);
    if (rc) return rc;
    SmallArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.n = n;
    sa.stop_cos2 = h->opt.precision == PSVD_PREC_FP64 ? 0.0 : 0x1p-30;
    sa.r = r;
    sa.K = h->K;
    sa.l = 0;
    sa.max_sweeps = h->opt.max_sweeps;
    sa.allow_fallback = (h->opt.flags & PSVD_OPT_NO_FALLBACK) ? 0 : 1;
    sa.d = h->d.as<double>();
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
    sa.sweeps = dstat + 1;
    const bool low_rank = h->ell > 0;
    const int ell = std::min(h->K, n);
    sa.skip_svd = low_rank ? 1 : 0;
    if (low_rank) {   // the batch's test matrix (n x ell, FP64 values) for the low-rank SVD of R
        std::vector<double> om((size_t)n * ell);
        gen_omega(h->opt.seed, h->batch, n, ell, 0, om.data());
        HIPCHK(h, h->lrom.ensure(om.size() * sizeof(double)));
        HIPCHK(h, h->lrwork.ensure(low_rank_work_doubles(n, n, ell) * sizeof(double)));
        HIPCHK(h, hipMemcpyAsync(h->lrom.p, om.data(), om.size() * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(h, hipStreamSynchronize(st));   // the host vector goes out of scope
    }
    {
        int pes = prof_begin(h, PSVD_KC_SMALL_SVD);
        HIPCHK(h, launch_small_det1(sa, st));
        prof_end(h, pes);
    }
    const int skipmask = DEV_FALLBACK | DEV_NONFINITE | DEV_BREAKDOWN;
    rc = nn_product_parts(h, Qin[0], qin, L.Xn, n, n, fp64, dstat, skipmask, PSVD_KC_NN);
    if (rc) return rc;
    rc = tn_product_parts(h, Q1[0], qg, nob, mbl, true, L.G2, dstat, skipmask);
    if (rc) return rc;
    {
        int pes = prof_begin(h, PSVD_KC_SMALL_SVD);
        HIPCHK(h, launch_small_det2(sa, st));
        if (low_rank) {
            // the low-rank SVD of R = R2 R1 (kept in G), T = R2^-1 U~_R for the lift
            LowRankArgs lr;
            std::memset(&lr, 0, sizeof(lr));
            lr.m = n;
            lr.n = n;
            lr.l = ell;
            lr.K = h->K;
            lr.A = L.G;
            lr.a_i = 1;
            lr.a_j = n;
            lr.Om = h->lrom.as<double>();
            lr.max_sweeps = h->opt.max_sweeps;
            lr.work = h->lrwork.as<double>();
            lr.U = L.sm_u;
            lr.ldu = n;
            lr.s = s_new;
            lr.post = 1;
            lr.post_R = L.G2;
            lr.T = L.T;
            lr.status = dstat;
            lr.sweeps = dstat + 1;
            HIPCHK(h, launch_low_rank_small(lr, st));
        }
        prof_end(h, pes);
    }
    // lift of every partition with the shared small factor (the eigen route
    // of a Cholesky breakdown lifts from the panel itself)
    rc = nn_product_parts(h, Q1[0], qn, L.T, n, rk, fp64, dstat, skipmask, PSVD_KC_LIFT);
    if (rc) return rc;
    rc = nn_product_parts(h, C[0], cn, L.T, n, rk, fp64, dstat, DEV_NONFINITE | DEV_BREAKDOWN, PSVD_KC_LIFT,
                          DEV_FALLBACK);
    if (rc) return rc;
    HIPCHK(h, hipEventRecord(h->ev1, st));
    HIPCHK(h, hipMemcpyAsync(h->status_host, dstat, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
    const int32_t sv = h->status_host[0];
    if (profiling(h)) prof_resolve(h);
    h->stats.last_sweeps = h->status_host[1];
    if (sv & DEV_FALLBACK) h->stats.fallbacks += 1;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) h->stats.last_update_ms = ms;
    if (int code = finish_status(h, sv)) return code;
    h->cur = nxt;
    h->r = rk;
    h->batch += 1;
    h->stats.batches += 1;
    h->stats.last_path = 0;
    return PSVD_OK;
}

int psvd_pstream_modes_ptr(const psvd_handle* h, int32_t part, const void** U, int64_t* ldu, int32_t* dtype) {
    if (!h || !U || h->parts.empty() || part < 0 || part >= (int32_t)h->parts.size()) return PSVD_E_INVAL;
    const int esz = h->u_dtype == PSVD_F64 ? 8 : 4;
    *U = (const char*)h->U[h->cur].p + (size_t)h->poff[part] * h->K * esz;
    if (ldu) *ldu = h->parts[part];
    if (dtype) *dtype = h->u_dtype;
    return PSVD_OK;
}

int psvd_pstream_modes(const psvd_handle* hc, int32_t part, void* U, int64_t ldu) {
    psvd_handle* h = const_cast<psvd_handle*>(hc);
    if (!h || h->parts.empty() || part < 0 || part >= (int32_t)h->parts.size()) return PSVD_E_INVAL;
    if (h->r == 0) return PSVD_OK;
    if (!U) return PSVD_E_INVAL;
    const int64_t Mi = h->parts[part];
    if (ldu < Mi) return fail(h, PSVD_E_SHAPE, "ldu < M_part");
    const int esz = h->u_dtype == PSVD_F64 ? 8 : 4;
    const char* src = (const char*)h->U[h->cur].p + (size_t)h->poff[part] * h->K * esz;
    HIPCHK(h, hipMemcpy2DAsync(U, ldu * esz, src, Mi * esz, Mi * esz, h->r, hipMemcpyDeviceToDevice, h->stream));
    return PSVD_OK;
}

}  // extern "C"
