"""GPU parity of the partitioned streaming SVD (the parallel variant of Sec. 3 on
row partitions of one GPU) against the FP64 oracle's partitioned stream.

Same seeded batches on both sides, split into uneven row partitions.  The
oracle initialises by APMOS and updates by local Householder QR per
partition, QR of the stacked R factors and SVD of the combined R; the library
sums the partitions' Gram partials into one Cholesky-QR2.  Tolerances: FP64
1e-10 (sigma), FP32 1e-4, as for the single-panel stream.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from conftest import sigma_rel_err, orth_err, align_signs, max_principal_angle

pytestmark = pytest.mark.gpu


def lib():
    import paper_2108_08845_amd as P
    return P


def split_gpu(b, sizes):
    """(N, M) contiguous tensor on the GPU -> row partitions as (M_i, N) column-major views."""
    out, o = [], 0
    for m in sizes:
        out.append(b[:, o: o + m].t())
        o += m
    return out


def split_np(A, sizes):
    out, o = [], 0
    for m in sizes:
        out.append(np.asfortranarray(A[o: o + m]))
        o += m
    return out


def run_both(w, sizes, precision, r_local, ff, low_rank=False, seed=0):
    P = lib()
    batches = synth.planted_stream(w)
    svd = P.PartitionedStreamingSVD(sizes, w.K, ff=ff, r_local=r_local, precision=precision, low_rank=low_rank,
                                    seed=seed)
    po = oracle.PartitionedStreamOracle(sizes, w.K, ff=ff, r_local=r_local, low_rank=low_rank, seed=seed)
    for b in batches:
        bg = b.to("cuda")
        svd.incorporate_data(split_gpu(bg, sizes))
        po.incorporate(split_np(synth.numpy_cm(b), sizes))
    return svd, po


@pytest.mark.parametrize("precision,dtype,tol", [("fp64", torch.float64, 1e-10), ("fp32", torch.float32, 1e-4)])
def test_pstream_matches_partitioned_oracle(precision, dtype, tol):
    # c1 shape (N = 64 per batch, K = 10, rank 20 > K: truncation loss) at 600
    # rows in four uneven partitions (one not a multiple of 4), ff = 0.9.
    w = synth.scaled(synth.c1_plain_fp64(), M=600, dtype=dtype)
    sizes = [150, 97, 203, 150]
    svd, po = run_both(w, sizes, precision, r_local=10, ff=0.9)
    s, s_ref = svd.singular_values, po.singular_values
    assert len(s) == len(s_ref) == w.K
    assert sigma_rel_err(s, s_ref) <= tol, sigma_rel_err(s, s_ref)
    U = svd.modes.double().cpu().numpy()
    assert orth_err(U) <= (1e-12 if precision == "fp64" else 1e-5)
    # the same sign rule on both sides: modes agree entry by entry, partition by partition
    etol = 1e-9 if precision == "fp64" else 2e-3
    for i in range(len(sizes)):
        Ui = svd.modes_part(i).double().cpu().numpy()
        assert np.abs(Ui - po.modes_part(i)).max() <= etol, i


@pytest.mark.parametrize("precision,dtype,tol", [("fp64", torch.float64, 1e-10), ("fp32", torch.float32, 1e-4)])
def test_pstream_low_rank_matches_partitioned_oracle(precision, dtype, tol):
    # The paper's placement of randomization: the SVD of W (APMOS
    # initialisation) and of every combined R factor by the low-rank SVD with a
    # K-column test matrix of (seed, batch), against the oracle's low-rank
    # partitioned stream on the same test matrices.
    w = synth.scaled(synth.c1_plain_fp64(), M=600, dtype=dtype)
    sizes = [150, 97, 203, 150]
    svd, po = run_both(w, sizes, precision, r_local=10, ff=0.9, low_rank=True, seed=11)
    s, s_ref = svd.singular_values, po.singular_values
    assert len(s) == len(s_ref) == w.K
    assert sigma_rel_err(s, s_ref) <= tol, sigma_rel_err(s, s_ref)
    U = svd.modes.double().cpu().numpy()
    assert orth_err(U) <= (1e-12 if precision == "fp64" else 1e-5)
    # the same sign rule on the same sketch basis: modes agree entry by entry
    etol = 1e-9 if precision == "fp64" else 2e-3
    for i in range(len(sizes)):
        Ui = svd.modes_part(i).double().cpu().numpy()
        assert np.abs(Ui - po.modes_part(i)).max() <= etol, i


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-4)])
def test_apmos_low_rank_matches_oracle(dtype, tol):
    # Algorithm 2 with the low-rank SVD of W (ell = 24 > K = 20, W of rank 40)
    w = synth.scaled(synth.c4_apmos(), partitions=8, part_min=500, part_max=3000, dtype=dtype)
    sizes = synth.partition_sizes(w)
    parts = synth.apmos_partitions(w, sizes=sizes)
    P = lib()
    ell, seed = 24, 17
    U, Lam, X = P.apmos_batched([p.to("cuda").t() for p in parts], w.local_rank, w.K, low_rank_ell=ell, seed=seed)
    Om = oracle.omega(seed, 0, len(parts) * w.local_rank, ell, oracle.PREC_F64)
    Uo, Lo, Xo = oracle.apmos([synth.numpy_cm(p) for p in parts], w.local_rank, w.K, omega=Om)
    assert sigma_rel_err(Lam, Lo) <= tol
    # same sketch basis and sign rule: X~ and the lifted modes agree directly
    assert np.abs(X - Xo).max() <= max(1e-9, 1e2 * tol)
    Ug = np.vstack([u.double().cpu().numpy() for u in U])
    assert np.abs(Ug - np.vstack(Uo)).max() <= max(1e-9, 1e2 * tol) * np.abs(np.vstack(Uo)).max()


def test_pstream_single_partition_equals_single_panel_stream():
    # P = 1 with r_local = N: the APMOS initialisation is the exact SVD of the
    # first batch (local rank 20 <= 64), so the stream equals the single-panel one.
    w = synth.scaled(synth.c1_plain_fp64(), M=800)
    batches = synth.planted_stream(w)
    P = lib()
    ps = P.PartitionedStreamingSVD([w.M], w.K, ff=0.95, r_local=w.N, precision="fp64")
    ss = P.StreamingSVD(w.M, w.K, ff=0.95, precision="fp64")
    for b in batches:
        bg = b.to("cuda")
        ps.incorporate_data([bg.t()])
        ss.incorporate_data(bg.t())
    assert sigma_rel_err(ps.singular_values, ss.singular_values) <= 1e-10
    Up = ps.modes.double().cpu().numpy()
    Us = ss.modes.double().cpu().numpy()
    assert np.abs(align_signs(Up, Us) - Us).max() <= 1e-8


def test_pstream_exact_low_rank():
    # rank 6 = K, ff = 1, no noise: every step is exact, the state is the SVD
    # of all batches (LAPACK), on uneven FP64 partitions.
    j = np.arange(6)
    w = synth.Workload("lowrank", M=900, N=30, batches=3, K=6, oversampling=0, power_iters=0, ff=1.0,
                       sigma=2.0 ** (-j / 2.0), noise=0.0, seed=5, dtype=torch.float64, randomized=False,
                       precision="fp64")
    sizes = [300, 275, 325]
    batches = synth.planted_stream(w)
    P = lib()
    ps = P.PartitionedStreamingSVD(sizes, w.K, ff=1.0, r_local=8, precision="fp64")
    for b in batches:
        ps.incorporate_data(split_gpu(b.to("cuda"), sizes))
    A = np.hstack([synth.numpy_cm(b) for b in batches])
    Ul, sl, _ = np.linalg.svd(A, full_matrices=False)
    assert sigma_rel_err(ps.singular_values, sl[:6]) <= 1e-11
    assert max_principal_angle(ps.modes.double().cpu().numpy(), Ul[:, :6]) <= 1e-9


def test_pstream_errors():
    import ctypes
    P = lib()
    from paper_2108_08845_amd import _lib
    w = synth.scaled(synth.c1_plain_fp64(), M=400)
    b = synth.planted_stream(w)[0].to("cuda")
    # a partition with fewer rows than the second panel has columns (K + N = 74)
    ps = P.PartitionedStreamingSVD([340, 60], w.K, ff=1.0, r_local=10, precision="fp64")
    ps.incorporate_data(split_gpu(b, [340, 60]))            # APMOS initialisation: fine
    with pytest.raises(P.PsvdError) as e:
        ps.incorporate_data(split_gpu(b, [340, 60]))
    assert e.value.code == -2                                # PSVD_E_SHAPE
    assert ps.rank == w.K                                    # state unchanged
    # single-panel calls are refused on a partitioned handle
    h = ps._h
    rc = _lib.load().psvd_incorporate_data(h, ctypes.c_void_p(b.data_ptr()), 400, 64, 400, _lib.PSVD_F64)
    assert rc == -9                                          # PSVD_E_STATE
    # FP32 data on an FP64 handle
    with pytest.raises(P.PsvdError):
        ps.incorporate_data([t.float() for t in split_gpu(b, [340, 60])])


def test_burgers_partitioned_stream_vs_serial():
    # The paper's first experiment at its size: Burgers snapshots of Eq. (13),
    # 16384 grid points x 800 snapshots (FP64), streamed in 8 batches of 100
    # with K = 20, ff = 1, on 4 row partitions against the single-panel stream
    # (serial) and the oracle's partitioned stream; modes 1 and 2 against the
    # SVD of the whole matrix (LAPACK).
    P = lib()
    u = synth.burgers_snapshots(16384, 800)              # (800, 16384): column-major 16384 x 800
    sizes = [4096] * 4
    K, nb = 20, 100
    ps = P.PartitionedStreamingSVD(sizes, K, ff=1.0, r_local=nb, precision="fp64")
    ss = P.StreamingSVD(16384, K, ff=1.0, precision="fp64")
    po = oracle.PartitionedStreamOracle(sizes, K, ff=1.0, r_local=nb)
    ug = u.to("cuda")
    A = synth.numpy_cm(u)
    for b in range(8):
        blk = ug[b * nb:(b + 1) * nb]                    # (nb, 16384) contiguous
        ps.incorporate_data(split_gpu(blk, sizes))
        ss.incorporate_data(blk.t())
        po.incorporate(split_np(np.asfortranarray(A[:, b * nb:(b + 1) * nb]), sizes))
    s_p, s_s, s_o = ps.singular_values, ss.singular_values, po.singular_values
    assert sigma_rel_err(s_p, s_o) <= 1e-10
    assert sigma_rel_err(s_p, s_s) <= 1e-10
    Up = ps.modes.double().cpu().numpy()
    Us = ss.modes.double().cpu().numpy()
    assert np.abs(Up[:, :2] - po.modes[:, :2]).max() <= 1e-9
    assert np.abs(align_signs(Up[:, :2], Us[:, :2]) - Us[:, :2]).max() <= 1e-9
    Ul, sl, _ = np.linalg.svd(A, full_matrices=False)
    assert sigma_rel_err(s_p[:2], sl[:2]) <= 1e-6           # truncation of the stream at K = 20
    assert np.abs(align_signs(Up[:, :2], Ul[:, :2]) - Ul[:, :2]).max() <= 1e-6
