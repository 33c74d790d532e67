// apmos.hip -- approximate partitioned method of snapshots (Algorithm 2,
// Eqs. 3-6) over many row partitions of uneven height on one GPU.
//
// Sequence, captured once into a hipGraph and replayed:
//   1. k_tn over a flattened (partition, row chunk) work list: G_i = A_i^T A_i
//      (method-of-snapshots form of the local SVD, FP64 accumulation),
//      partials summed per partition in a fixed order;
//   2. one work-group per partition: Jacobi eigen-decomposition of G_i,
//      W_i = V_i[:, :r] diag(sigma_i[:r])  (stored as W^T);
//   3. W W^T = sum_i W_i W_i^T (k_tn on W^T) and its Jacobi eigen-decomposition
//      -> X~, Lambda~ (the SVD of W of Eq. 5, truncated to K);
//   4. k_nn over the same work list: U_i = A_i X~ diag(1 / Lambda~)  (Eq. 6).
// With the paper's placement of randomization (psvd_apmos_low_rank), step 3 is
// the low-rank SVD of W instead (k_low_rank_small: Eqs. 7-11 on W with an
// ell-column Gaussian test matrix).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "kernels.h"

using namespace psvd;

namespace {

// Sign rule on the columns of W = the rows of W^T (rows x cols, leading
// dimension ld): each gets its largest-magnitude entry (lowest index on ties)
// non-negative.  The exact SVD of W does not see column signs (W W^T does not
// change); its low-rank SVD does (the sketch is W Om), so both sides fix them.
__global__ void k_wt_row_signs(double* Wt, int rows, int cols, int ld) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    double best = -1.0, v = 0.0;
    for (int k = 0; k < cols; ++k) {
        const double x = Wt[i + (size_t)k * ld];
        if (fabs(x) > best) {
            best = fabs(x);
            v = x;
        }
    }
    if (v < 0.0)
        for (int k = 0; k < cols; ++k) Wt[i + (size_t)k * ld] = -Wt[i + (size_t)k * ld];
}

struct ApmosWork {
    std::mutex mu;
    void* buf = nullptr;
    size_t bytes = 0;
    hipGraphExec_t exec = nullptr;
    // configuration the cached graph was captured for
    std::vector<int64_t> key;
    hipStream_t key_stream = nullptr;
};

ApmosWork& work_for_device() {
    static ApmosWork w[16];
    int dev = 0;
    (void)hipGetDevice(&dev);
    return w[dev & 15];
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// Algorithm 2 with the exact SVD of W (ell = 0) or its low-rank SVD with the
// test matrix of (seed, batch) with ell columns, FP64 values.
static int apmos_run(int32_t P, const void* const* A_parts, const int64_t* M_parts, const int64_t* ld_parts,
                     int64_t N, int32_t dtype, int32_t r, int32_t K, int32_t ell, uint64_t seed, int64_t batch,
                     void* const* U_parts, const int64_t* ldu_parts, double* Lambda, double* X, void* stream) {
    if (P < 1 || N < 1 || r < 1 || r > N || K < 1 || K > N || (int64_t)K > (int64_t)P * r || N > 4096)
        return PSVD_E_INVAL;
    if (ell < 0 || (ell > 0 && (ell < K || ell > N || (int64_t)ell > (int64_t)P * r))) return PSVD_E_INVAL;
    if (!A_parts || !M_parts || !ld_parts || !U_parts || !ldu_parts) return PSVD_E_INVAL;
    if (dtype != PSVD_F32 && dtype != PSVD_F64) return PSVD_E_DTYPE;
    int64_t Mtot = 0;
    for (int i = 0; i < P; ++i) {
        if (M_parts[i] < 1 || ld_parts[i] < M_parts[i] || ldu_parts[i] < M_parts[i] || !A_parts[i] || !U_parts[i])
            return PSVD_E_SHAPE;
        Mtot += M_parts[i];
    }
    hipStream_t st = (hipStream_t)stream;
    const bool fp64 = dtype == PSVD_F64;

    // Segments and the flattened work list.
    std::vector<PanelSeg> segs(P);
    for (int i = 0; i < P; ++i) {
        PanelSeg& s = segs[i];
        std::memset(&s, 0, sizeof(s));
        s.rows = M_parts[i];
        s.blk[0].ptr = A_parts[i];
        s.blk[0].ld = ld_parts[i];
        s.blk[0].dtype = dtype;
        s.blk[0].ncols = (int)N;
        s.nblk = 1;
        s.ncols = (int)N;
        s.out = U_parts[i];
        s.ldo = ldu_parts[i];
        s.out_dtype = dtype;
    }
    // float4 loads in the lift (k_nn_v): FP32 partitions, rows and leading
    // dimensions multiples of 4, 16-byte aligned bases
    bool tn_vec = true;   // 16-byte column loads in the Grams (k_tn_v), either dtype
    for (int i = 0; i < P; ++i)
        tn_vec = tn_vec && M_parts[i] % 4 == 0 && ld_parts[i] % 4 == 0 && ((uintptr_t)A_parts[i] & 15) == 0;
    const bool vec_all = !fp64 && tn_vec;
    const int mb = (int)((N + 63) / 64);
    const int nob = mb * (mb + 1) / 2;
    // about 2048 work-groups for the local Grams, one per (item, output block);
    // the whole-Gram kernel (N of 65..128) runs one per item and one per CU: at
    // most 256 items
    int64_t chunk = (mb == 2) ? chunk_for_items(M_parts, (int)P, 256)
                                        : std::max<int64_t>(64, ((Mtot / std::max(1, 2048 / nob) + 63) / 64) * 64);
    std::vector<WorkItem> items;
    std::vector<int32_t> seg_item0(P + 1);
    for (int i = 0; i < P; ++i) {
        seg_item0[i] = (int32_t)items.size();
        for (int64_t r0 = 0; r0 < M_parts[i]; r0 += chunk) {
            WorkItem w;
            w.seg = i;
            w.pad = 0;
            w.row0 = r0;
            w.row1 = std::min<int64_t>(r0 + chunk, M_parts[i]);
            items.push_back(w);
        }
    }
    seg_item0[P] = (int32_t)items.size();
    const int nitems = (int)items.size();
    // lift work list: finer chunks (one output block)
    int64_t lchunk = std::max<int64_t>(64, ((Mtot / 2048 + 63) / 64) * 64);
    std::vector<WorkItem> litems;
    for (int i = 0; i < P; ++i)
        for (int64_t r0 = 0; r0 < M_parts[i]; r0 += lchunk) {
            WorkItem w;
            w.seg = i;
            w.pad = 0;
            w.row0 = r0;
            w.row1 = std::min<int64_t>(r0 + lchunk, M_parts[i]);
            litems.push_back(w);
        }
    const int nlitems = (int)litems.size();
    const int pr = P * r;
    const int mbw = (int)((N + 63) / 64);

    // Workspace layout.
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off += align_up(b);
        return o;
    };
    size_t o_segs = take(sizeof(PanelSeg) * P);
    size_t o_items = take(sizeof(WorkItem) * nitems);
    size_t o_litems = take(sizeof(WorkItem) * nlitems);
    size_t o_si0 = take(sizeof(int32_t) * (P + 1));
    size_t o_part = take(sizeof(double) * (size_t)std::max(nitems, 1) * nob * TN_OB * TN_OB);
    size_t o_G = take(sizeof(double) * (size_t)P * N * N);
    size_t o_Wt = take(sizeof(double) * (size_t)pr * N);
    size_t o_WW = take(sizeof(double) * (size_t)N * N);
    size_t o_T = take(sizeof(double) * (size_t)N * K);
    size_t o_Lam = take(sizeof(double) * K);
    size_t o_X = take(sizeof(double) * (size_t)N * K);
    size_t o_vec = take(sizeof(double) * (size_t)P * (2 * N + 2) + 64);
    size_t o_ivec = take(sizeof(int32_t) * 3 * (size_t)P * N + 64);
    size_t o_stat = take(64);
    size_t o_wwpart = take(sizeof(double) * 2048 * (size_t)mbw * (mbw + 1) / 2 * TN_OB * TN_OB);
    size_t o_om = take(sizeof(double) * (size_t)pr * std::max(ell, 1));
    size_t o_lr = take(sizeof(double) * (ell > 0 ? low_rank_work_doubles((int)N, pr, ell) : 1));
    const size_t total = off;

    ApmosWork& W = work_for_device();
    std::lock_guard<std::mutex> lock(W.mu);
    hipError_t e = hipSuccess;
    if (total > W.bytes) {
        if (W.exec) {
            (void)hipGraphExecDestroy(W.exec);
            W.exec = nullptr;
        }
        if (W.buf) (void)hipFree(W.buf);
        W.buf = nullptr;
        W.bytes = 0;
        e = hipMalloc(&W.buf, total);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? PSVD_E_NOMEM : PSVD_E_DEVICE;
        W.bytes = total;
    }
    char* base = (char*)W.buf;
    PanelSeg* d_segs = (PanelSeg*)(base + o_segs);
    WorkItem* d_items = (WorkItem*)(base + o_items);
    WorkItem* d_litems = (WorkItem*)(base + o_litems);
    int32_t* d_si0 = (int32_t*)(base + o_si0);
    double* d_part = (double*)(base + o_part);
    double* d_G = (double*)(base + o_G);
    double* d_Wt = (double*)(base + o_Wt);
    double* d_WW = (double*)(base + o_WW);
    double* d_T = (double*)(base + o_T);
    double* d_Lam = (double*)(base + o_Lam);
    double* d_X = (double*)(base + o_X);
    double* d_vec = (double*)(base + o_vec);
    int32_t* d_ivec = (int32_t*)(base + o_ivec);
    int32_t* d_stat = (int32_t*)(base + o_stat);
    double* d_wwpart = (double*)(base + o_wwpart);
    double* d_om = (double*)(base + o_om);
    double* d_lr = (double*)(base + o_lr);

    // Descriptors (synchronous upload; the call is synchronous anyway).
    e = hipMemcpyAsync(d_segs, segs.data(), sizeof(PanelSeg) * P, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_items, items.data(), sizeof(WorkItem) * nitems, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_litems, litems.data(), sizeof(WorkItem) * nlitems, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_si0, seg_item0.data(), sizeof(int32_t) * (P + 1), hipMemcpyHostToDevice, st);
    std::vector<double> om;
    if (ell > 0) {
        om.resize((size_t)pr * ell);
        host_omega(seed, batch, pr, ell, 0, om.data());
        if (e == hipSuccess) e = hipMemcpyAsync(d_om, om.data(), sizeof(double) * om.size(), hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess) e = hipMemsetAsync(d_stat, 0, 64, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return PSVD_E_DEVICE;

    std::vector<int64_t> key = {P, N, r, K, dtype, nitems, nlitems, (int64_t)(uintptr_t)W.buf, (int64_t)total, ell,
                                (int64_t)vec_all};
    for (int i = 0; i < P; ++i) key.push_back(M_parts[i]);
    const bool reuse = W.exec && W.key == key && W.key_stream == st;

    auto enqueue = [&](hipStream_t s2) -> hipError_t {
            // 1. local Grams
            TnArgs ta;
            std::memset(&ta, 0, sizeof(ta));
            ta.lsegs = d_segs;
            ta.rsegs = d_segs;
            ta.lseg = segs[0];
            ta.rseg = segs[0];
            ta.items = d_items;
            ta.mbl = mb;
            ta.sym = 1;
            ta.part = d_part;
            ta.nob = nob;
            ta.vec = tn_vec ? 1 : 0;
            ta.dtype_all = dtype;
            hipError_t ce = launch_tn(true, ta, nitems, s2);
            TnReduceArgs tr;
            std::memset(&tr, 0, sizeof(tr));
            tr.part = d_part;
            tr.seg_item0 = d_si0;
            tr.nitems = nitems;
            tr.mbl = mb;
            tr.nob = nob;
            tr.nl = (int)N;
            tr.nr = (int)N;
            tr.sym = 1;
            tr.out = d_G;
            if (ce == hipSuccess) ce = launch_tn_reduce(tr, P, s2);
            // 2. local eigen-decompositions -> W^T
            ApmosLocalArgs la;
            la.G = d_G;
            la.Wt = d_Wt;
            la.N = (int)N;
            la.r = r;
            la.P = P;
            la.max_sweeps = 60;
            la.data_f32 = fp64 ? 0 : 1;
            la.vec = d_vec;
            la.ivec = d_ivec;
            la.status = d_stat;
            la.sweeps = d_stat + 1;
            if (ce == hipSuccess) ce = launch_apmos_local(la, s2);
            if (ce == hipSuccess) {
                hipLaunchKernelGGL(k_wt_row_signs, dim3((pr + 255) / 256), dim3(256), 0, s2, d_Wt, pr, (int)N, pr);
                ce = hipGetLastError();
            }
            // 3. the SVD of W: the low-rank SVD (Eqs. 7-11 on W = (W^T)^T) ...
            if (ell > 0) {
                LowRankArgs lr;
                std::memset(&lr, 0, sizeof(lr));
                lr.m = (int)N;
                lr.n = pr;
                lr.l = ell;
                lr.K = K;
                lr.A = d_Wt;          // W(i, j) = W^T(j, i) at d_Wt[j + i pr]
                lr.a_i = pr;
                lr.a_j = 1;
                lr.Om = d_om;
                lr.max_sweeps = 60;
                lr.work = d_lr;
                lr.U = d_X;
                lr.ldu = N;
                lr.s = d_Lam;
                lr.post = 2;
                lr.T = d_T;
                lr.status = d_stat;
                lr.sweeps = d_stat + 1;
                if (ce == hipSuccess) ce = launch_low_rank_small(lr, s2);
            }
            // ... or W W^T and its Jacobi eigen-decomposition
            PanelSeg ws;
            std::memset(&ws, 0, sizeof(ws));
            ws.rows = pr;
            ws.blk[0].ptr = d_Wt;
            ws.blk[0].ld = pr;
            ws.blk[0].dtype = PSVD_F64;
            ws.blk[0].ncols = (int)N;
            ws.nblk = 1;
            ws.ncols = (int)N;
            const int nobw = mbw * (mbw + 1) / 2;
            int64_t wchunk = std::max<int64_t>(64, ((pr / std::max(1, 1024 / nobw) + 63) / 64) * 64);
            int nwitems = (int)((pr + wchunk - 1) / wchunk);
            TnArgs wa;
            std::memset(&wa, 0, sizeof(wa));
            wa.lseg = ws;
            wa.rseg = ws;
            wa.chunk = wchunk;
            wa.mbl = mbw;
            wa.sym = 1;
            wa.part = d_wwpart;
            wa.nob = nobw;
            wa.vec = (pr % 4 == 0 && ((uintptr_t)d_Wt & 15) == 0) ? 1 : 0;
            wa.dtype_all = PSVD_F64;
            if (ce == hipSuccess && ell == 0) ce = launch_tn(true, wa, nwitems, s2);
            TnReduceArgs wr;
            std::memset(&wr, 0, sizeof(wr));
            wr.part = d_wwpart;
            wr.nitems = nwitems;
            wr.mbl = mbw;
            wr.nob = nobw;
            wr.nl = (int)N;
            wr.nr = (int)N;
            wr.sym = 1;
            wr.out = d_WW;
            if (ce == hipSuccess && ell == 0) ce = launch_tn_reduce(wr, 1, s2);
            ApmosGlobalArgs ga;
            ga.WW = d_WW;
            ga.N = (int)N;
            ga.K = K;
            ga.max_sweeps = 60;
            ga.T = d_T;
            ga.Lam = d_Lam;
            ga.X = d_X;
            ga.vec = d_vec;
            ga.ivec = d_ivec;
            ga.status = d_stat;
            ga.sweeps = d_stat + 1;
            if (ce == hipSuccess && ell == 0) ce = launch_apmos_global(ga, s2);
            // 4. lift over all partitions
            NnArgs na;
            std::memset(&na, 0, sizeof(na));
            na.seg = segs[0];
            na.segs = d_segs;
            na.items = d_litems;
            na.X = d_T;
            na.ldx = N;
            na.n = (int)N;
            na.nx = K;
            na.all_f32 = fp64 ? 0 : 1;
            na.vec_f32 = vec_all ? 1 : 0;
            na.vec16 = tn_vec ? 1 : 0;
            if (ce == hipSuccess) ce = launch_nn(fp64, na, nlitems, s2);
        return ce;
    };
    if (st == nullptr) {
        // The legacy default stream cannot be captured: enqueue directly.
        e = enqueue(st);
    } else {
        if (!reuse) {
            if (W.exec) {
                (void)hipGraphExecDestroy(W.exec);
                W.exec = nullptr;
            }
            hipGraph_t graph = nullptr;
            e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return PSVD_E_DEVICE;
            hipError_t ce = enqueue(st);
            e = hipStreamEndCapture(st, &graph);
            if (ce != hipSuccess || e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return PSVD_E_DEVICE;
            }
            e = hipGraphInstantiate(&W.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                W.exec = nullptr;
                return PSVD_E_DEVICE;
            }
            W.key = key;
            W.key_stream = st;
        }
        e = hipGraphLaunch(W.exec, st);
    }
    int32_t hstat[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(hstat, d_stat, sizeof(hstat), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && Lambda) e = hipMemcpyAsync(Lambda, d_Lam, sizeof(double) * K, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && X) e = hipMemcpyAsync(X, d_X, sizeof(double) * N * K, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? PSVD_E_NOMEM : PSVD_E_DEVICE;
    if (hstat[0] & DEV_NOCONV) return PSVD_E_NOCONV;
    if (hstat[0] & DEV_SMALL_LAMBDA) return PSVD_E_INVAL;
    return PSVD_OK;
}

extern "C" int psvd_apmos_batched(int32_t P, const void* const* A_parts, const int64_t* M_parts,
                                  const int64_t* ld_parts, int64_t N, int32_t dtype, int32_t r, int32_t K,
                                  void* const* U_parts, const int64_t* ldu_parts, double* Lambda, double* X,
                                  void* stream) {
    return apmos_run(P, A_parts, M_parts, ld_parts, N, dtype, r, K, 0, 0, 0, U_parts, ldu_parts, Lambda, X, stream);
}

extern "C" int psvd_apmos_low_rank(int32_t P, const void* const* A_parts, const int64_t* M_parts,
                                   const int64_t* ld_parts, int64_t N, int32_t dtype, int32_t r, int32_t K,
                                   int32_t ell, uint64_t seed, void* const* U_parts, const int64_t* ldu_parts,
                                   double* Lambda, double* X, void* stream) {
    if (ell < 1) return PSVD_E_INVAL;
    return apmos_run(P, A_parts, M_parts, ld_parts, N, dtype, r, K, ell, seed, 0, U_parts, ldu_parts, Lambda, X,
                     stream);
}

namespace psvd {
int apmos_internal(int32_t P, const void* const* A_parts, const int64_t* M_parts, const int64_t* ld_parts, int64_t N,
                   int32_t dtype, int32_t r, int32_t K, int32_t ell, uint64_t seed, int64_t batch,
                   void* const* U_parts, const int64_t* ldu_parts, double* Lambda, double* X, void* stream) {
    return apmos_run(P, A_parts, M_parts, ld_parts, N, dtype, r, K, ell, seed, batch, U_parts, ldu_parts, Lambda, X,
                     stream);
}
}  // namespace psvd
