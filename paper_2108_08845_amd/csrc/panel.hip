// panel.hip -- tall-skinny panel kernels on the gfx950 matrix cores.
//
// A "panel" is up to three column-major column blocks sharing rows (see
// PanelSeg).  Three kernels cover every pass over the tall data:
//   k_tn     Z = L^T R over row ranges (Gram C^T C, projection C^T Y, Y^T Y):
//            per-work-item partial sums, summed afterwards in a fixed order
//            (no floating-point atomics; results are run-to-run identical).
//   k_nn     Y = C X (sketch, lift U <- C T, APMOS lift), written per segment.
//   k_fused  P = C^T (C X) [and G = (C X)^T (C X)] in one read of C: the
//            row tile is staged once in LDS, Y_tile = C_tile X stays on chip
//            and feeds P += C_tile^T Y_tile (the range-finder passes).
// Row tiles are staged through LDS with coalesced column-segment loads; the
// next tile is prefetched into registers while the matrix cores work.
#include "kernels.h"

namespace psvd {

// ----------------------------------------------------------------------------
// Column pointer lookup (block-uniform per column).
// ----------------------------------------------------------------------------
struct ColRef {
    const char* base;  // column base
    int32_t dtype;
};

__device__ __forceinline__ ColRef col_ref(const PanelSeg& s, int c) {
    ColRef r{nullptr, PSVD_F32};
    int cc = c;
    for (int b = 0; b < s.nblk; ++b) {
        const PanelBlock& B = s.blk[b];
        if (cc < B.ncols) {
            int esz = B.dtype == PSVD_F64 ? 8 : 4;
            r.base = (const char*)B.ptr + (size_t)cc * (size_t)B.ld * esz;
            r.dtype = B.dtype;
            return r;
        }
        cc -= B.ncols;
    }
    return r;
}

__device__ __forceinline__ WorkItem get_item(const WorkItem* items, int64_t chunk, int64_t rows) {
    if (items) return items[blockIdx.x];
    WorkItem w;
    w.seg = 0;
    w.pad = 0;
    w.row0 = (int64_t)blockIdx.x * chunk;
    w.row1 = w.row0 + chunk < rows ? w.row0 + chunk : rows;
    return w;
}

__device__ __forceinline__ double ld_col(const ColRef& r, int64_t i) {
    return r.dtype == PSVD_F64 ? ((const double*)r.base)[i] : (double)((const float*)r.base)[i];
}

// ----------------------------------------------------------------------------
// k_tn: partial[item][ob] = L[rows, lcols]^T R[rows, rcols], 64 x 64 blocks.
// grid.x = work items, grid.y = output blocks (list in obl/obr).
// ----------------------------------------------------------------------------
constexpr int TN_TM = 64;
constexpr int TN_PAD = 1;


template <class CT>
__global__ __launch_bounds__(256) void k_tn(TnArgs a) {
    using MF = Mfma<CT>;
    using E = typename MF::elem;
    if (a.skip && (*a.skip & a.skip_mask)) return;
    __shared__ E Ls[TN_OB * (TN_TM + TN_PAD)];
    __shared__ E Rs[TN_OB * (TN_TM + TN_PAD)];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const WorkItem it = get_item(a.items, a.chunk, a.lseg.rows);
    const PanelSeg& L = a.lsegs ? a.lsegs[it.seg] : a.lseg;
    const PanelSeg& R = a.rsegs ? a.rsegs[it.seg] : a.rseg;
    const int ob = blockIdx.y;
    int obi, obj;
    block_coords(ob, a.mbl, a.sym, &obi, &obj);
    const int lc0 = obi * TN_OB, rc0 = obj * TN_OB;

    typename MF::acc acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = typename MF::acc{0, 0, 0, 0};

    // Per-thread load slots: 64 columns x 64 rows = 4096 elements per operand,
    // 16 per thread; consecutive threads read consecutive rows of a column.
    constexpr int PER = TN_OB * TN_TM / 256;
    double pl[PER], pr[PER];
    auto fetch = [&](int64_t r0) {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            int idx = e * 256 + tid;
            int c = idx / TN_TM, rr = idx % TN_TM;
            int64_t row = r0 + rr;
            double vl = 0.0, vr = 0.0;
            if (row < it.row1) {
                if (lc0 + c < L.ncols) vl = ld_col(col_ref(L, lc0 + c), row);
                if (rc0 + c < R.ncols) vr = ld_col(col_ref(R, rc0 + c), row);
            }
            pl[e] = vl;
            pr[e] = vr;
        }
    };
    fetch(it.row0);
    for (int64_t r0 = it.row0; r0 < it.row1; r0 += TN_TM) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            int idx = e * 256 + tid;
            int c = idx / TN_TM, rr = idx % TN_TM;
            Ls[c * (TN_TM + TN_PAD) + rr] = MF::from_double(pl[e]);
            Rs[c * (TN_TM + TN_PAD) + rr] = MF::from_double(pr[e]);
        }
        __syncthreads();
        if (r0 + TN_TM < it.row1) fetch(r0 + TN_TM);
        // wave w: output tile row block w, column blocks 0..3
#pragma unroll 4
        for (int k0 = 0; k0 < TN_TM; k0 += MF::KSTEP) {
            E av = Ls[(w * 16 + (lane & 15)) * (TN_TM + TN_PAD) + k0 + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                E bv = Rs[(j * 16 + (lane & 15)) * (TN_TM + TN_PAD) + k0 + (lane >> 4)];
                acc[j] = MF::mma(av, bv, acc[j]);
            }
        }
    }
    double* out = a.part + ((size_t)blockIdx.x * a.nob + ob) * (TN_OB * TN_OB);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int row = w * 16 + MF::row_of(lane, v);
            int col = j * 16 + (lane & 15);
            out[row + col * TN_OB] = (double)acc[j][v];
        }
}

// Sum the partials of all items of each segment in item order and scatter the
// 64 x 64 blocks into dense FP64 outputs out[seg] (nl x nr, ld nl); Gram
// (sym != 0): the lower block triangle is mirrored from the upper one.

__global__ __launch_bounds__(256) void k_tn_reduce(TnReduceArgs a) {
    if (a.skip && (*a.skip & a.skip_mask)) return;
    const int seg = blockIdx.y, ob = blockIdx.z;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= TN_OB * TN_OB) return;
    const int i = e % TN_OB, j = e / TN_OB;
    int obi, obj;
    block_coords(ob, a.mbl, a.sym, &obi, &obj);
    const int gi = obi * TN_OB + i, gj = obj * TN_OB + j;
    if (gi >= a.nl || gj >= a.nr) return;
    double s = 0.0;
    const int it0 = a.seg_item0 ? a.seg_item0[seg] : 0;
    const int it1 = a.seg_item0 ? a.seg_item0[seg + 1] : a.nitems;
    for (int it = it0; it < it1; ++it)
        s += a.part[((size_t)it * a.nob + ob) * (TN_OB * TN_OB) + e];
    double* o = a.out + (size_t)seg * a.nl * a.nr;
    if (a.row_scale && gi < a.nscale) s *= a.row_scale[gi];
    o[gi + (size_t)gj * a.nl] = s;
    if (a.sym && obi != obj) o[gj + (size_t)gi * a.nl] = s;
}

// ----------------------------------------------------------------------------
// k_nn: out[seg rows, ocols] = C[rows, :] X[:, ocols] (+ optional row scale).
// grid.x = work items, grid.y = output column blocks of 64.
// ----------------------------------------------------------------------------
constexpr int NN_TM = 64;
constexpr int NN_KC = 32;
constexpr int NN_OB = 64;


template <class CT>
__global__ __launch_bounds__(256) void k_nn(NnArgs a) {
    using MF = Mfma<CT>;
    using E = typename MF::elem;
    if (a.skip && (*a.skip & a.skip_mask)) return;
    if (a.skip && a.need_mask && !(*a.skip & a.need_mask)) return;
    __shared__ E Cs[NN_KC * (NN_TM + 1)];
    __shared__ E Xs[NN_OB * (NN_KC + 1)];
    __shared__ double Os[NN_OB * (NN_TM + 1)];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const WorkItem it = get_item(a.items, a.chunk, a.seg.rows);
    const PanelSeg& S = a.segs ? a.segs[it.seg] : a.seg;
    const int oc0 = blockIdx.y * NN_OB;
    for (int64_t r0 = it.row0; r0 < it.row1; r0 += NN_TM) {
        typename MF::acc acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = typename MF::acc{0, 0, 0, 0};
        for (int k0 = 0; k0 < a.n; k0 += NN_KC) {
            __syncthreads();
            // C chunk: 32 columns x 64 rows (8 per thread)
#pragma unroll
            for (int e = 0; e < NN_KC * NN_TM / 256; ++e) {
                int idx = e * 256 + tid;
                int c = idx / NN_TM, rr = idx % NN_TM;
                int64_t row = r0 + rr;
                double v = 0.0;
                if (row < it.row1 && k0 + c < a.n) v = ld_col(col_ref(S, k0 + c), row);
                Cs[c * (NN_TM + 1) + rr] = MF::from_double(v);
            }
            // X chunk: 32 rows x 64 columns
#pragma unroll
            for (int e = 0; e < NN_KC * NN_OB / 256; ++e) {
                int idx = e * 256 + tid;
                int k = idx % NN_KC, j = idx / NN_KC;
                double v = 0.0;
                if (k0 + k < a.n && oc0 + j < a.nx) v = a.X[(k0 + k) + (int64_t)(oc0 + j) * a.ldx];
                Xs[j * (NN_KC + 1) + k] = MF::from_double(v);
            }
            __syncthreads();
            // wave w: output row block w (16 rows), column blocks 0..3
#pragma unroll
            for (int kk = 0; kk < NN_KC; kk += MF::KSTEP) {
                E av = Cs[(kk + (lane >> 4)) * (NN_TM + 1) + w * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    E bv = Xs[(j * 16 + (lane & 15)) * (NN_KC + 1) + kk + (lane >> 4)];
                    acc[j] = MF::mma(av, bv, acc[j]);
                }
            }
        }
        // Stage the output tile through LDS for coalesced column stores.
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int row = w * 16 + MF::row_of(lane, v);
                int col = j * 16 + (lane & 15);
                Os[col * (NN_TM + 1) + row] = (double)acc[j][v];
            }
        __syncthreads();
        for (int idx = tid; idx < NN_OB * NN_TM; idx += 256) {
            int rr = idx % NN_TM, j = idx / NN_TM;
            int64_t row = r0 + rr;
            if (row < it.row1 && oc0 + j < a.nx) {
                double v = Os[j * (NN_TM + 1) + rr];
                if (a.row_scale && row < a.nscale) v *= a.row_scale[row];
                size_t o = (size_t)row + (size_t)(oc0 + j) * (size_t)S.ldo;
                if (S.out_dtype == PSVD_F64) {
                    double* po = (double*)S.out + o;
                    *po = a.accumulate ? *po + v : v;
                } else {
                    float* po = (float*)S.out + o;
                    *po = a.accumulate ? (float)((double)*po + v) : (float)v;
                }
            }
        }
    }
}

// ----------------------------------------------------------------------------
// k_fused: P = C^T (C X) and optionally G = (C X)^T (C X), one read of C.
// CT = bf16_t (power passes of the mixed precision) or float.
// One column block of LB = 64 columns of X per work-group (grid.y > 1 splits
// wider sketches; consecutive blocks of a row range run on the same XCD).
// ----------------------------------------------------------------------------


template <class MF>
__device__ __forceinline__ typename MF::frag lds_frag(const typename MF::elem* p) {
    if constexpr (MF::KPL == 1) {
        return *p;
    } else {
        uint64_t u = *(const uint64_t*)p;  // 4 bf16, 8-byte aligned by construction
        return __builtin_bit_cast(s4_t, u);
    }
}

// Column base pointer (FP32 panel) of column c.
__device__ __forceinline__ const float* fcol(const PanelSeg& s, int c) {
    int cc = c;
    for (int b = 0; b < s.nblk; ++b) {
        if (cc < s.blk[b].ncols) return (const float*)s.blk[b].ptr + (size_t)cc * (size_t)s.blk[b].ld;
        cc -= s.blk[b].ncols;
    }
    return nullptr;
}

// Work-group of 512 threads (8 waves).  Tile = TM rows x np columns of the
// panel.  Each thread moves float4 column segments: TPC = TM / 4 threads per
// column, CPR = 512 / TPC columns per round.
//   MODE 0: P += C^T (C X)             (power pass)
//   MODE 1: P and G = (C X)^T (C X)    (final pass; FP32 only)
//   MODE 2: out = C X                  (lift; FP32 only)
template <class CT, int TM, int NRB, bool VEC, int MODE>
__global__ __launch_bounds__(512) void k_fused(FusedArgs a) {
    using MF = Mfma<CT>;
    using E = typename MF::elem;
    constexpr int NT = 512;
    constexpr int KPL = MF::KPL;
    constexpr int KSTEP = MF::KSTEP;
    constexpr bool ROWCOPY = (KPL > 1);
    constexpr int TPC = TM / 4;
    constexpr int CPR = NT / TPC;
    constexpr int NPMAX = NRB * 8 * 16;
    constexpr int RMAX = (NPMAX + CPR - 1) / CPR;
    extern __shared__ __align__(16) unsigned char smem[];
    const int np = a.np;
    const int ldX = np + 4;
    const int ldC = TM + 4;
    const int ldR = np + 4;
    const int ldY = TM + 4;
    E* Xs = (E*)smem;
    E* Cs = Xs + (size_t)FU_LB * ldX;
    E* Cr = Cs + (size_t)np * ldC;
    E* Ys = Cr + (ROWCOPY ? (size_t)TM * ldR : 0);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int b = blockIdx.x;
    const int xcd = b & 7, local = b >> 3;
    const int lb = local % a.nlb;
    const int wg = (local / a.nlb) * 8 + xcd;
    if (wg >= a.nwg) return;
    const int c0 = lb * FU_LB;

    for (int idx = tid; idx < FU_LB * np; idx += NT) {
        int k = idx % np, j = idx / np;
        double v = 0.0;
        if (k < a.n && c0 + j < a.lx) v = a.X[k + (int64_t)(c0 + j) * a.ldx];
        Xs[j * ldX + k] = MF::from_double(v);
    }

    const int nrb = np / 16;
    typename MF::acc accP[MODE == 2 ? 1 : NRB * 4];
#pragma unroll
    for (int t = 0; t < (MODE == 2 ? 1 : NRB * 4); ++t) accP[t] = typename MF::acc{0, 0, 0, 0};
    d4_t accG[2];
    accG[0] = d4_t{0, 0, 0, 0};
    accG[1] = d4_t{0, 0, 0, 0};

    const int rounds = (np + CPR - 1) / CPR;
    const int tsub = tid % TPC, tcol = tid / TPC;
    f4_t pf[RMAX];
    auto fetch = [&](int64_t t) {
        const int64_t row = t * TM + tsub * 4;
#pragma unroll
        for (int rr = 0; rr < RMAX; ++rr) {
            f4_t v = f4_t{0.f, 0.f, 0.f, 0.f};
            const int c = rr * CPR + tcol;
            if (rr < rounds && c < a.n) {
                const float* p = fcol(a.seg, c);
                if (VEC && row + 3 < a.seg.rows) {
                    v = *(const f4_t*)(p + row);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (row + q < a.seg.rows) v[q] = p[row + q];
                }
            }
            pf[rr] = v;
        }
    };

    int64_t t = wg;
    if (t < a.tiles) fetch(t);
    for (; t < a.tiles; t += a.nwg) {
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < RMAX; ++rr) {
            const int c = rr * CPR + tcol;
            if (rr < rounds && c < np) {
                if constexpr (sizeof(E) == 4) {
                    *(f4_t*)&Cs[c * ldC + tsub * 4] = pf[rr];
                } else {
                    uint16_t h0 = MF::from_float(pf[rr][0]), h1 = MF::from_float(pf[rr][1]);
                    uint16_t h2 = MF::from_float(pf[rr][2]), h3 = MF::from_float(pf[rr][3]);
                    uint64_t pk = (uint64_t)h0 | ((uint64_t)h1 << 16) | ((uint64_t)h2 << 32) | ((uint64_t)h3 << 48);
                    *(uint64_t*)&Cs[c * ldC + tsub * 4] = pk;
                    if (ROWCOPY) {
                        Cr[(tsub * 4 + 0) * ldR + c] = h0;
                        Cr[(tsub * 4 + 1) * ldR + c] = h1;
                        Cr[(tsub * 4 + 2) * ldR + c] = h2;
                        Cr[(tsub * 4 + 3) * ldR + c] = h3;
                    }
                }
            }
        }
        __syncthreads();
        if (t + a.nwg < a.tiles) fetch(t + a.nwg);

        // Phase A: Y_tile (TM x 64) = C_tile X_blk.  (TM/16) x 4 output tiles over 8 waves.
        constexpr int YT = (TM / 16) * 4;
        for (int yt = w; yt < YT; yt += 8) {
            const int ib = yt >> 2, jb = yt & 3;
            // Four interleaved accumulators keep consecutive matrix-core ops independent.
            typename MF::acc acc4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc4[u] = typename MF::acc{0, 0, 0, 0};
            for (int k0 = 0; k0 < np; k0 += 4 * KSTEP) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int kk = k0 + u * KSTEP;
                    if (kk < np) {
                        typename MF::frag bv =
                            lds_frag<MF>(&Xs[(jb * 16 + (lane & 15)) * ldX + kk + (lane >> 4) * KPL]);
                        typename MF::frag av;
                        if constexpr (KPL == 1) av = Cs[(kk + (lane >> 4)) * ldC + ib * 16 + (lane & 15)];
                        else av = lds_frag<MF>(&Cr[(ib * 16 + (lane & 15)) * ldR + kk + (lane >> 4) * KPL]);
                        acc4[u] = MF::mma(av, bv, acc4[u]);
                    }
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = ib * 16 + MF::row_of(lane, v);
                const int col = jb * 16 + (lane & 15);
                Ys[col * ldY + row] = MF::from_acc((acc4[0][v] + acc4[1][v]) + (acc4[2][v] + acc4[3][v]));
            }
        }
        __syncthreads();

        if (MODE == 2 || (MODE == 1 && a.yout != nullptr)) {
            // Y_tile -> out (lift) or the copy of Y (final pass), float4 column segments, j < lx
            float* obase = MODE == 2 ? (float*)a.seg.out : a.yout;
            const int64_t ldo = MODE == 2 ? a.seg.ldo : a.ldy;
            const int64_t row = t * TM + tsub * 4;
            for (int j = tcol; j < FU_LB; j += CPR) {
                if (c0 + j >= a.lx) continue;
                f4_t v = *(const f4_t*)&Ys[j * ldY + tsub * 4];
                float* o = obase + (size_t)(c0 + j) * (size_t)ldo;
                if (VEC && row + 3 < a.seg.rows) {
                    *(f4_t*)(o + row) = v;
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (row + q < a.seg.rows) o[row + q] = v[q];
                }
            }
        }
        if constexpr (MODE != 2) {
            // Phase B: P (np x 64) += C_tile^T Y_tile; wave w owns row blocks w, w+8, ...
#pragma unroll
            for (int k0 = 0; k0 < TM; k0 += KSTEP) {
                typename MF::frag bvs[4];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    bvs[j] = lds_frag<MF>(&Ys[(j * 16 + (lane & 15)) * ldY + k0 + (lane >> 4) * KPL]);
#pragma unroll
                for (int q = 0; q < NRB; ++q) {
                    const int rb = w + 8 * q;
                    if (rb < nrb) {
                        typename MF::frag av =
                            lds_frag<MF>(&Cs[(rb * 16 + (lane & 15)) * ldC + k0 + (lane >> 4) * KPL]);
#pragma unroll
                        for (int j = 0; j < 4; ++j) accP[q * 4 + j] = MF::mma(av, bvs[j], accP[q * 4 + j]);
                    }
                }
            }
            if constexpr (MODE == 1) {
                // G (64 x 64) += Y^T Y in FP64 on the FP32 values; wave w: row block w/2, col blocks (w%2)*2 + {0,1}
                const int gi = w >> 1, gj0 = (w & 1) * 2;
#pragma unroll
                for (int k0 = 0; k0 < TM; k0 += 4) {
                    double av = (double)*(const float*)&Ys[(gi * 16 + (lane & 15)) * ldY + k0 + (lane >> 4)];
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        double bv = (double)*(const float*)&Ys[((gj0 + j) * 16 + (lane & 15)) * ldY + k0 + (lane >> 4)];
                        accG[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, accG[j], 0, 0, 0);
                    }
                }
            }
        }
    }
    if constexpr (MODE != 2) {
        float* outP = a.partP + ((size_t)wg * a.nlb + lb) * (size_t)np * FU_LB;
#pragma unroll
        for (int q = 0; q < NRB; ++q) {
            const int rb = w + 8 * q;
            if (rb < nrb) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = rb * 16 + MF::row_of(lane, v);
                        const int col = j * 16 + (lane & 15);
                        outP[row + (size_t)col * np] = accP[q * 4 + j][v];
                    }
            }
        }
    }
    if constexpr (MODE == 1) {
        double* outG = a.partG + (size_t)wg * FU_LB * FU_LB;
        const int gi = w >> 1, gj0 = (w & 1) * 2;
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = gi * 16 + Mfma<double>::row_of(lane, v);
                const int col = (gj0 + j) * 16 + (lane & 15);
                outG[row + col * FU_LB] = accG[j][v];
            }
    }
}

// ----------------------------------------------------------------------------
// k_sketch_bf16: the BF16 power pass P += C^T (C X) with the 16x16x32 BF16
// matrix-core instruction.  X (np x 64) lives in registers for the whole
// launch; every tile is read once from HBM, converted to BF16 and written to
// LDS twice (column-major for C^T Y, row-major for C X) with packed stores:
// each thread moves a 4 x 4 block (four float4 column segments).
// ----------------------------------------------------------------------------
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef short s8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf8_t lds_b128(const uint16_t* p) {
    return __builtin_bit_cast(bf8_t, *(const s8_t*)p);   // 16-byte aligned by construction
}

template <int TM, int NRB, bool VEC>
__global__ __launch_bounds__(512) void k_sketch_bf16(FusedArgs a) {
    constexpr int NT = 512;
    constexpr int JW = TM == 64 ? 2 : 1;            // column blocks of Y per wave in phase A
    constexpr int NPMAX = NRB * 128;
    constexpr int KS = NPMAX / 32;                  // k-steps of phase A
    constexpr int RG = TM / 4;                      // row groups of 4
    constexpr int CGR = NT / RG;                    // column groups (of 4) per round
    constexpr int RMAX = (NPMAX / 4 + CGR - 1) / CGR;
    extern __shared__ __align__(16) unsigned char smem[];
    const int np = a.np;
    const int ldC = TM + 8;
    const int ldR = np + 8;
    const int ldY = TM + 8;
    uint16_t* Cs = (uint16_t*)smem;                 // np x TM, column-major
    uint16_t* Cr = Cs + (size_t)np * ldC;           // TM x np, row-major
    uint16_t* Ys = Cr + (size_t)TM * ldR;           // 64 x TM, column-major

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int b = blockIdx.x;
    const int xcd = b & 7, local = b >> 3;
    const int lb = local % a.nlb;
    const int wg = (local / a.nlb) * 8 + xcd;
    if (wg >= a.nwg) return;
    const int c0 = lb * FU_LB;

    // Phase-A unit of this wave: row block ib, column blocks jb0 .. jb0 + JW - 1.
    const int ib = TM == 64 ? (w & 3) : (TM == 32 ? (w & 1) : 0);
    const int jb0 = TM == 64 ? (w >> 2) * 2 : (TM == 32 ? (w >> 1) : w);
    const bool a_active = (TM >= 32) || (w < 4);
    bf8_t xf[JW][KS];
#pragma unroll
    for (int c = 0; c < JW; ++c)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            bf8_t v;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int k = ks * 32 + 8 * (lane >> 4) + q;
                const int j = c0 + (jb0 + c) * 16 + (lane & 15);
                double x = (k < a.n && j < a.lx) ? a.X[k + (int64_t)j * a.ldx] : 0.0;
                v[q] = __builtin_bit_cast(__bf16, f32_to_bf16_rne((float)x));
            }
            xf[c][ks] = v;
        }

    const int nrb = np / 16;
    f4_t accP[NRB * 4];
#pragma unroll
    for (int t = 0; t < NRB * 4; ++t) accP[t] = f4_t{0.f, 0.f, 0.f, 0.f};

    const int ncg = np / 4;
    const int rounds = (ncg + CGR - 1) / CGR;
    const int rg = tid % RG, cgl = tid / RG;
    f4_t pf[RMAX][4];
    auto fetch = [&](int64_t t) {
        const int64_t row = t * TM + rg * 4;
#pragma unroll
        for (int rr = 0; rr < RMAX; ++rr) {
            const int cg = rr * CGR + cgl;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                f4_t v = f4_t{0.f, 0.f, 0.f, 0.f};
                const int c = cg * 4 + q;
                if (rr < rounds && c < a.n) {
                    const float* p = fcol(a.seg, c);
                    if (VEC && row + 3 < a.seg.rows) {
                        v = *(const f4_t*)(p + row);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (row + e < a.seg.rows) v[e] = p[row + e];
                    }
                }
                pf[rr][q] = v;
            }
        }
    };

    int64_t t = wg;
    if (t < a.tiles) fetch(t);
    for (; t < a.tiles; t += a.nwg) {
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < RMAX; ++rr) {
            const int cg = rr * CGR + cgl;
            if (rr < rounds && cg < ncg) {
                uint16_t h[4][4];   // [column q][row e]
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int e = 0; e < 4; ++e) h[q][e] = f32_to_bf16_rne(pf[rr][q][e]);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint64_t pk = (uint64_t)h[q][0] | ((uint64_t)h[q][1] << 16) | ((uint64_t)h[q][2] << 32) |
                                  ((uint64_t)h[q][3] << 48);
                    *(uint64_t*)&Cs[(cg * 4 + q) * ldC + rg * 4] = pk;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    uint64_t pk = (uint64_t)h[0][e] | ((uint64_t)h[1][e] << 16) | ((uint64_t)h[2][e] << 32) |
                                  ((uint64_t)h[3][e] << 48);
                    *(uint64_t*)&Cr[(rg * 4 + e) * ldR + cg * 4] = pk;
                }
            }
        }
        __syncthreads();
        if (t + a.nwg < a.tiles) fetch(t + a.nwg);

        // Phase A: Y_tile = C_tile X (X fragments in registers).
        if (a_active) {
            // Two interleaved accumulators per column block (independent consecutive ops).
            f4_t accY[JW][2];
#pragma unroll
            for (int c = 0; c < JW; ++c) accY[c][0] = accY[c][1] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                if (ks * 32 < np) {
                    bf8_t av = lds_b128(&Cr[(ib * 16 + (lane & 15)) * ldR + ks * 32 + 8 * (lane >> 4)]);
#pragma unroll
                    for (int c = 0; c < JW; ++c)
                        accY[c][ks & 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, xf[c][ks], accY[c][ks & 1], 0, 0, 0);
                }
            }
#pragma unroll
            for (int c = 0; c < JW; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = ib * 16 + 4 * (lane >> 4) + v;
                    const int col = (jb0 + c) * 16 + (lane & 15);
                    Ys[col * ldY + row] = f32_to_bf16_rne(accY[c][0][v] + accY[c][1][v]);
                }
        }
        __syncthreads();

        // Phase B: P (np x 64) += C_tile^T Y_tile; wave w owns row blocks w, w + 8, ...
#pragma unroll
        for (int ks = 0; ks < TM / 32; ++ks) {
            bf8_t bvs[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) bvs[j] = lds_b128(&Ys[(j * 16 + (lane & 15)) * ldY + ks * 32 + 8 * (lane >> 4)]);
#pragma unroll
            for (int q = 0; q < NRB; ++q) {
                const int rb = w + 8 * q;
                if (rb < nrb) {
                    bf8_t av = lds_b128(&Cs[(rb * 16 + (lane & 15)) * ldC + ks * 32 + 8 * (lane >> 4)]);
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        accP[q * 4 + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bvs[j], accP[q * 4 + j], 0, 0, 0);
                }
            }
        }
    }
    float* outP = a.partP + ((size_t)wg * a.nlb + lb) * (size_t)np * FU_LB;
#pragma unroll
    for (int q = 0; q < NRB; ++q) {
        const int rb = w + 8 * q;
        if (rb < nrb) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rb * 16 + 4 * (lane >> 4) + v;
                    const int col = j * 16 + (lane & 15);
                    outP[row + (size_t)col * np] = accP[q * 4 + j][v];
                }
        }
    }
}

size_t sketch_lds_bytes(int tm, int np) {
    return ((size_t)np * (tm + 8) + (size_t)tm * (np + 8) + (size_t)FU_LB * (tm + 8)) * 2;
}

int sketch_pick_tm(int np) {
    if (np > 640 || np % 32) return 0;
    for (int tm : {64, 32})
        if (sketch_lds_bytes(tm, np) <= 160 * 1024 && (np <= 384 || tm == 32)) return tm;
    return 0;
}

template <int TM, int NRB, bool VEC>
static hipError_t launch_sketch_k(const FusedArgs& a, hipStream_t st) {
    size_t lds = sketch_lds_bytes(TM, a.np);
    int blocks = ((a.nwg + 7) / 8) * 8 * a.nlb;
    hipError_t e = hipFuncSetAttribute((const void*)k_sketch_bf16<TM, NRB, VEC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sketch_bf16<TM, NRB, VEC>), dim3(blocks), dim3(512), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_sketch_bf16(const FusedArgs& a, hipStream_t st) {
    const bool v = a.vec != 0;
    if (a.tm == 64 && a.np <= 384) return v ? launch_sketch_k<64, 3, true>(a, st) : launch_sketch_k<64, 3, false>(a, st);
    if (a.tm == 32 && a.np <= 384) return v ? launch_sketch_k<32, 3, true>(a, st) : launch_sketch_k<32, 3, false>(a, st);
    if (a.tm == 32 && a.np <= 640) return v ? launch_sketch_k<32, 5, true>(a, st) : launch_sketch_k<32, 5, false>(a, st);
    return hipErrorInvalidValue;
}

// Fixed-order FP64 sum of the fused partials: P (n x lx, ld n) and G (lx x lx).

// 32 outputs per block, 8 threads per output each summing every 8th partial;
// the 8 sums are combined in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_fused_reduce(FusedReduceArgs a) {
    __shared__ double red[8][33];
    const int lane_o = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const int64_t e = (int64_t)blockIdx.x * 32 + lane_o;
    const int64_t totP = (int64_t)a.n * a.lx;
    const int64_t tot = totP + (a.want_g ? (int64_t)a.lx * a.lx : 0);
    double s = 0.0;
    if (e < totP) {
        const int i = (int)(e % a.n), j = (int)(e / a.n);
        const int lb = j / FU_LB, jj = j % FU_LB;
        const size_t stride = (size_t)a.nlb * a.np * FU_LB;
        const float* p = a.partP + (size_t)lb * a.np * FU_LB + i + (size_t)jj * a.np;
        for (int g = grp; g < a.nwg; g += 8) s += (double)p[(size_t)g * stride];
    } else if (e < tot) {
        const int64_t f = e - totP;
        const int i = (int)(f % a.lx), j = (int)(f / a.lx);
        const double* p = a.partG + i + (size_t)j * FU_LB;
        for (int g = grp; g < a.nwg; g += 8) s += p[(size_t)g * FU_LB * FU_LB];
    }
    red[grp][lane_o] = s;
    __syncthreads();
    if (grp == 0 && e < tot) {
        double t = 0.0;
        for (int q = 0; q < 8; ++q) t += red[q][lane_o];
        if (e < totP) {
            const int i = (int)(e % a.n), j = (int)(e / a.n);
            if (a.row_scale && i < a.nscale) t *= a.row_scale[i];
            a.P[i + (size_t)j * a.n] = t;
        } else {
            const int64_t f = e - totP;
            a.G[(f % a.lx) + (size_t)(f / a.lx) * a.lx] = t;
        }
    }
}

// ----------------------------------------------------------------------------
// Host launchers.
// ----------------------------------------------------------------------------
size_t fused_lds_bytes(int ct_bytes, bool rowcopy, int tm, int np) {
    size_t e = (size_t)FU_LB * (np + 4) + (size_t)np * (tm + 4) + (rowcopy ? (size_t)tm * (np + 4) : 0) +
               (size_t)FU_LB * (tm + 4);
    return e * ct_bytes;
}

hipError_t launch_tn(bool fp64, const TnArgs& a, int nitems, hipStream_t st) {
    dim3 grid(nitems, a.nob);
    if (fp64) hipLaunchKernelGGL(k_tn<double>, grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL(k_tn<float>, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_tn_reduce(const TnReduceArgs& a, int nseg, hipStream_t st) {
    dim3 grid((TN_OB * TN_OB + 255) / 256, nseg, a.nob);
    hipLaunchKernelGGL(k_tn_reduce, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_nn(bool fp64, const NnArgs& a, int nitems, hipStream_t st) {
    dim3 grid(nitems, (a.nx + NN_OB - 1) / NN_OB);
    if (fp64) hipLaunchKernelGGL(k_nn<double>, grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL(k_nn<float>, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

template <class CT, int TM, int NRB, bool VEC, int MODE>
static hipError_t launch_fused_k(const FusedArgs& a, size_t lds, hipStream_t st) {
    int blocks = ((a.nwg + 7) / 8) * 8 * a.nlb;
    hipError_t e = hipFuncSetAttribute((const void*)k_fused<CT, TM, NRB, VEC, MODE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fused<CT, TM, NRB, VEC, MODE>), dim3(blocks), dim3(512), lds, st, a);
    return hipGetLastError();
}

template <class CT, int TM, bool VEC, int MODE>
static hipError_t launch_fused_n(const FusedArgs& a, size_t lds, hipStream_t st) {
    if (a.np <= 128) return launch_fused_k<CT, TM, 1, VEC, MODE>(a, lds, st);
    if (a.np <= 384) return launch_fused_k<CT, TM, 3, VEC, MODE>(a, lds, st);
    if (a.np <= 640) return launch_fused_k<CT, TM, 5, VEC, MODE>(a, lds, st);
    return hipErrorInvalidValue;
}

template <class CT, bool VEC, int MODE>
static hipError_t launch_fused_m(const FusedArgs& a, size_t lds, hipStream_t st) {
    if (a.tm == 16) return launch_fused_n<CT, 16, VEC, MODE>(a, lds, st);
    if (a.tm == 32) return launch_fused_n<CT, 32, VEC, MODE>(a, lds, st);
    return launch_fused_n<CT, 64, VEC, MODE>(a, lds, st);
}

// Largest tile height whose LDS footprint fits one CU (0: none fits).
int fused_pick_tm(bool bf16, int np) {
    if (np > 640) return 0;
    for (int tm : {64, 32, 16})
        if (fused_lds_bytes(bf16 ? 2 : 4, bf16, tm, np) <= 160 * 1024) return tm;
    return 0;
}

bool fused_fits(bool bf16, int tm, int np) { return tm > 0 && np <= 640 && fused_lds_bytes(bf16 ? 2 : 4, bf16, tm, np) <= 160 * 1024; }

hipError_t launch_fused(bool bf16, int mode, const FusedArgs& a, hipStream_t st) {
    size_t lds = fused_lds_bytes(bf16 ? 2 : 4, bf16, a.tm, a.np);
    bool vec = a.vec != 0;
    if (bf16) {
        if (mode != 0) return hipErrorInvalidValue;
        return vec ? launch_fused_m<bf16_t, true, 0>(a, lds, st) : launch_fused_m<bf16_t, false, 0>(a, lds, st);
    }
    if (mode == 0) return vec ? launch_fused_m<float, true, 0>(a, lds, st) : launch_fused_m<float, false, 0>(a, lds, st);
    if (mode == 1) return vec ? launch_fused_m<float, true, 1>(a, lds, st) : launch_fused_m<float, false, 1>(a, lds, st);
    return vec ? launch_fused_m<float, true, 2>(a, lds, st) : launch_fused_m<float, false, 2>(a, lds, st);
}

hipError_t launch_fused_reduce(const FusedReduceArgs& a, hipStream_t st) {
    int64_t tot = (int64_t)a.n * a.lx + (a.want_g ? (int64_t)a.lx * a.lx : 0);
    dim3 grid((unsigned)((tot + 31) / 32));
    hipLaunchKernelGGL(k_fused_reduce, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace psvd
