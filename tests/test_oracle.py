"""Pins of the FP64 CPU oracle against what the mathematics fixes (no GPU).

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms, invariants, special cases that reduce to
a LAPACK routine (numpy.linalg), brute-force definitions on small inputs and
finite differences.  A plausible slip in the oracle (dropped term, wrong
sign, transposed operand, wrong index) fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from conftest import sigma_rel_err, max_principal_angle, orth_err, align_signs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rng(seed=0):
    return np.random.default_rng(seed)


def planted(M, N, sigma, seed=0, noise=0.0):
    g = rng(seed)
    Phi, _ = np.linalg.qr(g.standard_normal((M, len(sigma))))
    C, _ = np.linalg.qr(g.standard_normal((N, len(sigma))))
    A = Phi @ np.diag(sigma) @ C.T
    if noise:
        A = A + noise * g.standard_normal((M, N))
    return np.asfortranarray(A), Phi, C


# ----------------------------------------------------------------------------
# Test-matrix generator (Philox4x32-10 + Box-Muller)
# ----------------------------------------------------------------------------

def test_philox_known_answers():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(x, 16) for x in line.split()])
    assert len(rows) == 3
    for r in rows:
        assert oracle.philox4x32_10(r[0:4], r[4:6]) == r[6:10]


def test_omega_box_muller_definition():
    # Element pairs (2t, 2t+1) are the Box-Muller transform of the two 53-bit
    # uniforms built from Philox call t with counter (t, 0, batch, 0).
    seed, batch, n, ell = 0x1234_5678_9ABC, 3, 7, 3
    Om = oracle.omega(seed, batch, n, ell, oracle.PREC_F64).ravel(order="F")
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for t in range((n * ell + 1) // 2):
        x = oracle.philox4x32_10([t, 0, batch, 0], key)
        u1 = ((x[0] >> 5) * 2.0 ** 26 + (x[1] >> 6)) * 2.0 ** -53
        u2 = ((x[2] >> 5) * 2.0 ** 26 + (x[3] >> 6)) * 2.0 ** -53
        rad = math.sqrt(-2.0 * math.log(1.0 - u1))
        z = [rad * math.cos(2 * math.pi * u2), rad * math.sin(2 * math.pi * u2)]
        for h in range(2):
            e = 2 * t + h
            if e < n * ell:
                assert abs(Om[e] - z[h]) <= 1e-15 * max(1.0, abs(z[h]))


def test_omega_statistics_and_rounding():
    Om = oracle.omega(7, 0, 400, 250, oracle.PREC_F64)
    assert abs(Om.mean()) < 0.01 and abs(Om.std() - 1.0) < 0.01
    # Different batches and seeds give different draws; the same key repeats.
    assert not np.array_equal(Om, oracle.omega(7, 1, 400, 250, oracle.PREC_F64))
    assert not np.array_equal(Om, oracle.omega(8, 0, 400, 250, oracle.PREC_F64))
    assert np.array_equal(Om, oracle.omega(7, 0, 400, 250, oracle.PREC_F64))
    # float32: round-to-nearest of the double.
    O32 = oracle.omega(7, 0, 400, 250, oracle.PREC_F32)
    assert np.array_equal(O32, Om.astype(np.float32).astype(np.float64))
    # bfloat16: the float32 value rounded to 8 significant bits, ties to even.
    Ob = oracle.omega(7, 0, 400, 250, oracle.PREC_BF16)
    f = O32.astype(np.float32).view(np.uint32)
    lsb = (f >> 16) & 1
    ref = ((f + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32).view(np.float32).astype(np.float64)
    assert np.array_equal(Ob, ref)
    assert np.all((Ob.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)


# ----------------------------------------------------------------------------
# Householder QR
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("m,n", [(200, 50), (64, 64), (1000, 1), (37, 20)])
def test_hhqr_invariants_and_lapack(m, n):
    A = rng(m + n).standard_normal((m, n))
    Q, R = oracle.hhqr(A)
    tol = 1e-14 * math.sqrt(n)
    assert np.linalg.norm(A - Q @ R) / np.linalg.norm(A) <= tol
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= tol * 10
    assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)
    # Uniqueness of the positive-diagonal factorisation against LAPACK.
    Ql, Rl = np.linalg.qr(A)
    sgn = np.sign(np.diag(Rl))
    sgn[sgn == 0] = 1
    Ql, Rl = Ql * sgn, (Rl.T * sgn).T
    assert np.abs(R - Rl).max() <= 1e-12 * np.abs(Rl).max()
    assert np.abs(Q - Ql).max() <= 1e-12


def test_hhqr_rank_deficient_and_zero_column():
    g = rng(3)
    A = g.standard_normal((50, 6))
    A[:, 3] = A[:, 1] * 2.0          # dependent column
    A[:, 5] = 0.0                    # zero column
    Q, R = oracle.hhqr(A)
    assert np.linalg.norm(A - Q @ R) <= 1e-13 * np.linalg.norm(A)
    assert np.linalg.norm(Q.T @ Q - np.eye(6)) <= 1e-13
    assert abs(R[3, 3]) <= 1e-13 and abs(R[5, 5]) <= 1e-13


# ----------------------------------------------------------------------------
# One-sided Jacobi SVD
# ----------------------------------------------------------------------------

def test_jacobi_closed_forms():
    # Diagonal matrix: singular values are |d| sorted, vectors are +-e_i.
    d = np.array([0.5, -3.0, 2.0, 0.0, 1.0])
    U, s, V = oracle.jacobi_svd(np.diag(d))
    assert np.allclose(s, [3.0, 2.0, 1.0, 0.5, 0.0], atol=0, rtol=0)
    # Rank one sigma u v^T.
    g = rng(1)
    u = g.standard_normal(30); u /= np.linalg.norm(u)
    v = g.standard_normal(8); v /= np.linalg.norm(v)
    U, s, V = oracle.jacobi_svd(4.5 * np.outer(u, v))
    assert abs(s[0] - 4.5) <= 1e-14 * 4.5 and np.all(s[1:] <= 1e-14)
    assert abs(abs(U[:, 0] @ u) - 1) <= 1e-14 and abs(abs(V[:, 0] @ v) - 1) <= 1e-14
    # 2x2 closed form: singular values of [[a, b], [0, c]].
    a, b, c = 3.0, 4.0, 2.0
    fro2, det = a * a + b * b + c * c, a * c
    s1 = math.sqrt((fro2 + math.sqrt(fro2 ** 2 - 4 * det * det)) / 2)
    s2 = abs(det) / s1
    _, s, _ = oracle.jacobi_svd(np.array([[a, b], [0.0, c]]))
    assert abs(s[0] - s1) <= 1e-15 * s1 and abs(s[1] - s2) <= 1e-14 * s2


@pytest.mark.parametrize("m,n", [(200, 50), (50, 50), (120, 7)])
def test_jacobi_vs_lapack(m, n):
    A = rng(10 + n).standard_normal((m, n)) @ np.diag(np.logspace(0, -6, n))
    U, s, V = oracle.jacobi_svd(A)
    sl = np.linalg.svd(A, compute_uv=False)
    assert sigma_rel_err(s, sl) <= 1e-13 * 10
    assert np.linalg.norm(A - (U * s) @ V.T) / np.linalg.norm(A) <= 1e-13
    assert orth_err(U) <= 1e-13 and orth_err(V) <= 1e-13
    assert np.all(np.diff(s) <= 0)


def test_jacobi_sweep_limit_reports_nonconvergence():
    A = rng(2).standard_normal((40, 30))
    with pytest.raises(RuntimeError, match="-6"):
        oracle.jacobi_svd(A, max_sweeps=1)


# ----------------------------------------------------------------------------
# Deterministic streaming (Algorithm 1)
# ----------------------------------------------------------------------------

def test_planted_spectrum_recovered_exactly():
    sig = 2.0 ** (-np.arange(12) / 2.0)
    A, Phi, _ = planted(600, 40, sig, seed=5)
    so = oracle.StreamOracle(600, 12).incorporate(A)
    assert sigma_rel_err(so.singular_values, sig) <= 1e-12
    assert max_principal_angle(so.modes, Phi) <= 1e-11


@pytest.mark.parametrize("nb", [1, 2, 4])
def test_stream_ff1_equals_batch_svd(nb):
    # No truncation loss (K >= total rank): any batch split gives the SVD of the concatenation.
    sig = np.linspace(2.0, 0.2, 8)
    A, _, _ = planted(500, 64, sig, seed=11)
    so = oracle.StreamOracle(500, 10, ff=1.0)
    for b in np.split(np.arange(64), nb):
        so.incorporate(A[:, b])
    Ul, sl, _ = np.linalg.svd(A, full_matrices=False)
    assert sigma_rel_err(so.singular_values[:8], sl[:8]) <= 1e-12
    assert max_principal_angle(so.modes[:, :8], Ul[:, :8]) <= 1e-10


def test_stream_forget_factor_closed_form():
    # With no truncation loss, batch i's weight after the last batch is ff^(last-i).
    ff = 0.9
    sig = np.linspace(3.0, 0.5, 6)
    A, _, _ = planted(300, 30, sig, seed=12)
    parts = [A[:, :10], A[:, 10:20], A[:, 20:]]
    so = oracle.StreamOracle(300, 12, ff=ff)
    for p in parts:
        so.incorporate(p)
    W = np.hstack([ff ** 2 * parts[0], ff * parts[1], parts[2]])
    Ul, sl, _ = np.linalg.svd(W, full_matrices=False)
    assert sigma_rel_err(so.singular_values[:6], sl[:6]) <= 1e-12
    assert max_principal_angle(so.modes[:, :6], Ul[:, :6]) <= 1e-10


def test_stream_each_step_is_topk_svd_of_panel():
    # With truncation loss (rank 20 > K = 10) every step of Algorithm 1 is the
    # rank-K truncated SVD of its panel [ff U diag(s) | A_i]; pin each step
    # against LAPACK on the panel built from the oracle's own previous state.
    w = synth.scaled(synth.c1_plain_fp64(), M=512)
    batches = [synth.numpy_cm(t) for t in synth.planted_stream(w)]
    so = oracle.StreamOracle(w.M, w.K, ff=0.8)
    for A in batches:
        C = A if so.r == 0 else np.hstack([0.8 * so.modes * so.singular_values, A])
        so.incorporate(A)
        Ul, sl, _ = np.linalg.svd(C, full_matrices=False)
        k = so.r
        assert k == min(w.K, C.shape[1])
        assert sigma_rel_err(so.singular_values, sl[:k]) <= 1e-12
        U = align_signs(so.modes, Ul[:, :k])
        assert np.abs(U - Ul[:, :k]).max() <= 1e-9
        assert orth_err(so.modes) <= 1e-13


def test_stream_sign_rule():
    # Each column of the small left factor has its largest-magnitude entry positive.
    A, _, _ = planted(200, 20, np.linspace(1, 0.1, 5), seed=4)
    so = oracle.StreamOracle(200, 5).incorporate(A[:, :10]).incorporate(A[:, 10:])
    Ut = so.last_small_u
    for j in range(Ut.shape[1]):
        col = Ut[:, j]
        assert col[np.argmax(np.abs(col))] > 0


def test_stream_metamorphic():
    g = rng(21)
    A = np.asfortranarray(g.standard_normal((150, 12)) @ np.diag(np.logspace(0, -2, 12)))
    base = oracle.StreamOracle(150, 6).incorporate(A[:, :6]).incorporate(A[:, 6:])
    # Scaling the data scales the singular values.
    sc = oracle.StreamOracle(150, 6).incorporate(3 * A[:, :6]).incorporate(3 * A[:, 6:])
    assert sigma_rel_err(sc.singular_values, 3 * base.singular_values) <= 1e-13
    # A right orthogonal transform of a batch leaves the left data unchanged.
    O, _ = np.linalg.qr(g.standard_normal((6, 6)))
    rt = oracle.StreamOracle(150, 6).incorporate(A[:, :6] @ O).incorporate(A[:, 6:] @ O)
    assert sigma_rel_err(rt.singular_values, base.singular_values) <= 1e-12
    assert max_principal_angle(rt.modes[:, :4], base.modes[:, :4]) <= 1e-9
    # A row permutation permutes the rows of U.
    p = g.permutation(150)
    pm = oracle.StreamOracle(150, 6).incorporate(A[p, :6]).incorporate(A[p, 6:])
    assert sigma_rel_err(pm.singular_values, base.singular_values) <= 1e-12
    assert np.abs(align_signs(pm.modes, base.modes[p]) - base.modes[p]).max() <= 1e-9


def test_stream_empty_batch_is_noop():
    so = oracle.StreamOracle(50, 3).incorporate(rng(0).standard_normal((50, 4)))
    U, s = so.modes.copy(), so.singular_values.copy()
    so.incorporate(np.zeros((50, 0)))
    assert np.array_equal(U, so.modes) and np.array_equal(s, so.singular_values)


# ----------------------------------------------------------------------------
# Randomized streaming (Eqs. (7)-(11))
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("q", [0, 1, 2])
def test_randomized_exact_when_rank_fits_sketch(q):
    # rank(C) <= ell: Q spans range(C) for any Gaussian test matrix, so the
    # randomized step is exact whatever q is.
    sig = np.logspace(0, -1, 9)
    A, Phi, _ = planted(400, 60, sig, seed=31)
    so = oracle.StreamOracle(400, 8, oversampling=4, power_iters=q, randomized=True, seed=5)
    so.incorporate(A)
    assert sigma_rel_err(so.singular_values, sig[:8]) <= 1e-12
    assert max_principal_angle(so.modes, Phi[:, :8]) <= 1e-10


@pytest.mark.parametrize("q", [0, 1, 2])
def test_randomized_equals_ritz_of_power_sketch(q):
    # Closed form of what the range finder computes: Q = orth((C C^T)^q C Omega)
    # and (U, s) = the top-K SVD of Q Q^T C.  Rank(C) > ell, so q matters.
    g = rng(40 + q)
    M, N, K, p = 300, 40, 6, 4
    C = np.asfortranarray(g.standard_normal((M, N)) @ np.diag(np.linspace(1.0, 0.3, N)))
    so = oracle.StreamOracle(M, K, oversampling=p, power_iters=q, randomized=True, seed=9)
    Om = oracle.omega(9, 0, N, K + p, oracle.PREC_F64)
    so.incorporate(C)
    Y = C @ Om
    for _ in range(q):
        Y = C @ (C.T @ Y)
    Q, _ = np.linalg.qr(Y)
    Ub, sb, _ = np.linalg.svd(Q.T @ C, full_matrices=False)
    assert sigma_rel_err(so.singular_values, sb[:K]) <= 1e-11
    U = align_signs(so.modes, Q @ Ub[:, :K])
    assert np.abs(U - Q @ Ub[:, :K]).max() <= 1e-9


def test_randomized_power_iterations_reduce_error():
    # Halko-Martinsson-Tropp: power iterations sharpen the sketch on a slowly
    # decaying spectrum (statistical sanity check, fixed seeds).
    g = rng(50)
    M, N, K, p = 500, 120, 10, 5
    A = np.asfortranarray(g.standard_normal((M, N)) @ np.diag(1.0 / np.arange(1, N + 1) ** 0.5))
    s_true = np.linalg.svd(A, compute_uv=False)[:K]
    errs = []
    for q in (0, 1, 2):
        so = oracle.StreamOracle(M, K, oversampling=p, power_iters=q, randomized=True, seed=3).incorporate(A)
        errs.append(sigma_rel_err(so.singular_values, s_true))
    assert errs[0] > errs[1] > errs[2]
    assert np.all(so.singular_values <= s_true * (1 + 1e-12))   # Ritz values interlace


def test_randomized_falls_back_when_sketch_is_wide():
    A, _, _ = planted(100, 10, np.linspace(1, 0.1, 10), seed=2)
    a = oracle.StreamOracle(100, 5, oversampling=8, randomized=True).incorporate(A)
    b = oracle.StreamOracle(100, 5).incorporate(A)
    assert np.array_equal(a.singular_values, b.singular_values)


# ----------------------------------------------------------------------------
# APMOS (Algorithm 2)
# ----------------------------------------------------------------------------

def test_apmos_exact_when_local_rank_fits():
    w = synth.scaled(synth.c4_apmos(), partitions=5, part_min=300, part_max=700, N=48)
    sizes = synth.partition_sizes(w)
    parts = [synth.numpy_cm(t) for t in synth.apmos_partitions(w, sizes=sizes)]
    A = np.vstack(parts)
    Ul, sl, _ = np.linalg.svd(A, full_matrices=False)
    U, Lam, X = oracle.apmos(parts, 40, 20)           # r = 40 >= local rank 40
    assert sigma_rel_err(Lam, sl[:20]) <= 1e-11
    Us = np.vstack(U)
    assert max_principal_angle(Us, Ul[:, :20]) <= 1e-9
    assert orth_err(Us) <= 1e-10


def test_apmos_single_partition_is_svd():
    A = np.asfortranarray(rng(6).standard_normal((400, 30)) @ np.diag(np.logspace(0, -3, 30)))
    Ul, sl, _ = np.linalg.svd(A, full_matrices=False)
    U, Lam, X = oracle.apmos([A], 30, 10)
    assert sigma_rel_err(Lam, sl[:10]) <= 1e-12
    assert np.abs(align_signs(U[0], Ul[:, :10]) - Ul[:, :10]).max() <= 1e-10
    # The lift divides by Lambda: U^i = A^i X diag(1/Lambda).
    assert np.allclose(U[0], A @ X / Lam, atol=1e-14)


def test_apmos_truncated_local_rank_is_gram_of_W():
    # With r < local rank, the global step is the SVD of W = [V_i S_i]: check X, Lambda against
    # the eigen-decomposition of W W^T built from LAPACK local SVDs.
    g = rng(8)
    parts = [np.asfortranarray(g.standard_normal((m, 16)) @ np.diag(np.logspace(0, -2, 16))) for m in (90, 120, 70)]
    r, K = 5, 6
    Ws = []
    for Ai in parts:
        _, si, Vt = np.linalg.svd(Ai, full_matrices=False)
        Ws.append(Vt.T[:, :r] * si[:r])
    W = np.hstack(Ws)
    Xl, ll, _ = np.linalg.svd(W, full_matrices=False)
    U, Lam, X = oracle.apmos(parts, r, K)
    assert sigma_rel_err(Lam, ll[:K]) <= 1e-12
    assert np.abs(align_signs(X, Xl[:, :K]) - Xl[:, :K]).max() <= 1e-10


# ----------------------------------------------------------------------------
# The paper's placement of randomization: the low-rank SVD (Eqs. (7)-(11)) of
# W in Algorithm 2 and of the combined R factor of the partitioned update
# ----------------------------------------------------------------------------

def test_low_rank_svd_exact_when_rank_fits_sketch():
    # rank 5 <= ell: range(A Om) = range(A), so the low-rank SVD is the SVD
    sig = np.array([3.0, 1.5, 0.9, 0.4, 0.2])
    A, _, _ = planted(60, 45, sig, seed=31)
    Ul, sl, _ = np.linalg.svd(A, full_matrices=False)
    for ell in (5, 7):
        U, s = oracle.low_rank_svd(A, 5, oracle.omega(3, 0, 45, ell, oracle.PREC_F64))
        assert sigma_rel_err(s, sl[:5]) <= 1e-12
        assert max_principal_angle(U, Ul[:, :5]) <= 1e-10
        assert orth_err(U) <= 1e-13


def test_low_rank_svd_is_ritz_of_the_sketch():
    # general A, ell < rank: the values are the singular values of Q^T A with
    # Q an orthonormal basis of A Om (LAPACK), so none exceeds the true one
    g = rng(32)
    A = np.asfortranarray(g.standard_normal((50, 40)) @ np.diag(np.logspace(0, -2, 40)))
    Om = oracle.omega(5, 2, 40, 8, oracle.PREC_F64)
    U, s = oracle.low_rank_svd(A, 6, Om)
    Q, _ = np.linalg.qr(A @ Om)
    Ub, sb, _ = np.linalg.svd(Q.T @ A)
    sl = np.linalg.svd(A, compute_uv=False)
    assert len(s) == 6
    assert sigma_rel_err(s, sb[:6]) <= 1e-12
    assert max_principal_angle(U, Q @ Ub[:, :6]) <= 1e-10
    assert np.all(s <= sl[:6] * (1 + 1e-12))
    assert s[0] < sl[0]                       # a sketch of 8 columns misses part of the top mode


def test_apmos_low_rank_exact_when_W_rank_fits_sketch():
    # W has rank 20 (the planted spectrum has 20 modes), ell = K = 20: the
    # low-rank SVD of W is exact, so APMOS matches its exact form
    w = synth.scaled(synth.c4_apmos(), partitions=4, part_min=200, part_max=500, N=48, sigma=2.0 ** (-np.arange(20) / 3.0),
                     dtype=torch.float64)
    parts = [synth.numpy_cm(t) for t in synth.apmos_partitions(w)]
    U, Lam, X = oracle.apmos(parts, 25, 20)
    Om = oracle.omega(7, 0, 4 * 25, 20, oracle.PREC_F64)
    U2, Lam2, X2 = oracle.apmos(parts, 25, 20, omega=Om)
    assert sigma_rel_err(Lam2, Lam) <= 1e-11
    assert np.abs(align_signs(X2, X) - X).max() <= 1e-9
    assert max_principal_angle(np.vstack(U2), np.vstack(U)) <= 1e-9


def test_apmos_low_rank_is_low_rank_svd_of_W():
    # Truncated local ranks and ell < rank(W): X~ and Lambda~ are the low-rank
    # SVD of W = [V_i S_i] with the same test matrix.  Partitions [diag(d_i); 0]
    # make W known without any SVD: the local right singular vectors are the
    # coordinate vectors of the r largest d_i (positive, descending), so
    # W_i = [d_i,pi(1) e_pi(1), ..., d_i,pi(r) e_pi(r)]; Q, B = Q^T W and the SVD
    # of B are taken with LAPACK.
    g = rng(33)
    N, r, K, ell = 16, 5, 4, 6
    parts, Ws = [], []
    for m in (90, 120, 70):
        d = g.uniform(0.1, 2.0, N)
        Ai = np.zeros((m, N))
        Ai[:N, :N] = np.diag(d)
        parts.append(np.asfortranarray(Ai))
        Wi = np.zeros((N, r))
        for j, c in enumerate(np.argsort(-d, kind="stable")[:r]):
            Wi[c, j] = d[c]
        Ws.append(Wi)
    W = np.hstack(Ws)
    Om = oracle.omega(9, 0, 3 * r, ell, oracle.PREC_F64)
    Q, _ = np.linalg.qr(W @ Om)
    Ub, sb, _ = np.linalg.svd(Q.T @ W)
    U, Lam, X = oracle.apmos(parts, r, K, omega=Om)
    assert sigma_rel_err(Lam, sb[:K]) <= 1e-12
    assert np.abs(align_signs(X, (Q @ Ub)[:, :K]) - (Q @ Ub)[:, :K]).max() <= 1e-10
    sw = np.linalg.svd(W, compute_uv=False)
    assert np.all(Lam <= sw[:K] * (1 + 1e-12))          # Ritz values of a sketch of W


def test_pstream_low_rank_exact_when_rank_fits():
    # rank 6 = K = ell, ff = 1, no local truncation loss: the low-rank SVDs of
    # W and of every combined R are exact, so the stream is the SVD of the
    # concatenation (LAPACK)
    sig = np.linspace(3.0, 0.4, 6)
    A, _, _ = planted(700, 40, sig, seed=34)
    sizes = [150, 250, 300]
    po = oracle.PartitionedStreamOracle(sizes, 6, ff=1.0, r_local=10, low_rank=True, seed=5)
    for b in np.split(np.arange(40), 4):
        po.incorporate(_split_rows(A[:, b], sizes))
    Ul, sl, _ = np.linalg.svd(A, full_matrices=False)
    assert sigma_rel_err(po.singular_values[:6], sl[:6]) <= 1e-12
    assert max_principal_angle(po.modes[:, :6], Ul[:, :6]) <= 1e-10


def test_pstream_low_rank_update_is_low_rank_svd_of_R():
    # one low-rank partitioned update from a given state: the kept values are
    # the low-rank SVD (same test matrix) of the R factor of the stacked panel
    w = synth.scaled(synth.c1_plain_fp64(), M=600)
    batches = [synth.numpy_cm(t) for t in synth.planted_stream(w)]
    sizes = [120, 97, 200, 183]
    po = oracle.PartitionedStreamOracle(sizes, w.K, ff=0.9, low_rank=True, seed=4)
    po.incorporate(_split_rows(batches[0], sizes))
    U0, s0 = po.modes.copy(), po.singular_values.copy()
    C = np.hstack([0.9 * U0 * s0, batches[1]])
    _, R = np.linalg.qr(C)
    R = np.diag(np.sign(np.diag(R))) @ R                 # non-negative diagonal
    Om = oracle.omega(4, 1, C.shape[1], w.K, oracle.PREC_F64)
    Q, _ = np.linalg.qr(R @ Om)
    sb = np.linalg.svd(Q.T @ R, compute_uv=False)
    po.incorporate(_split_rows(batches[1], sizes))
    assert sigma_rel_err(po.singular_values, sb[:w.K]) <= 1e-11
    assert orth_err(po.modes) <= 1e-12


# ----------------------------------------------------------------------------
# Loss and gradient
# ----------------------------------------------------------------------------

# ----------------------------------------------------------------------------
# Burgers snapshots (the paper's first experiment, Eq. (13))
# ----------------------------------------------------------------------------

def test_burgers_generator_matches_closed_form():
    # a few entries of the generator against the closed form written directly
    u = synth.numpy_cm(synth.burgers_snapshots(513, 41))
    Re, t0 = 1000.0, math.exp(1000.0 / 8.0)
    for xi, ti in [(0, 0), (100, 0), (256, 7), (400, 40), (512, 20)]:
        x, t = xi / 512.0, 2.0 * ti / 40.0
        ref = (x / (t + 1.0)) / (1.0 + math.sqrt((t + 1.0) / t0) * math.exp(Re * x * x / (4.0 * t + 4.0)))
        assert abs(u[xi, ti] - ref) <= 1e-15 * max(1.0, abs(ref))
    assert np.isfinite(u).all() and u[0].max() == 0.0   # u(0, t) = 0


def test_burgers_partitioned_modes_match_serial():
    # Serial SVD (LAPACK) against APMOS over 4 row partitions with the
    # paper's local truncation r1 = 50: the first two modes agree.
    A = synth.numpy_cm(synth.burgers_snapshots(4096, 200))
    Ul, sl, _ = np.linalg.svd(A, full_matrices=False)
    parts = [np.asfortranarray(p) for p in np.split(A, 4)]
    Us, lam, _ = oracle.apmos(parts, 50, 5)
    Ua = np.vstack(Us)
    assert sigma_rel_err(lam[:2], sl[:2]) <= 1e-12
    assert np.abs(align_signs(Ua[:, :2], Ul[:, :2]) - Ul[:, :2]).max() <= 1e-12


# ----------------------------------------------------------------------------
# Partitioned streaming (the parallel variant of Sec. 3 on row partitions)
# ----------------------------------------------------------------------------

def _split_rows(A, sizes):
    out, o = [], 0
    for m in sizes:
        out.append(np.asfortranarray(A[o: o + m]))
        o += m
    return out


def test_pstream_update_equals_serial_update():
    # One partitioned update from the same state as the serial oracle: the
    # stacked R factors re-factored give the R of the whole panel, so the
    # update is the serial Algorithm 1 step of the stacked panel.  Pinned
    # against the serial oracle, itself pinned to LAPACK above; uneven
    # partitions, truncation loss (rank 20 > K = 10) and ff < 1.
    w = synth.scaled(synth.c1_plain_fp64(), M=600)
    batches = [synth.numpy_cm(t) for t in synth.planted_stream(w)]
    sizes = [120, 97, 200, 183]
    so = oracle.StreamOracle(w.M, w.K, ff=0.9)
    so.incorporate(batches[0])
    po = oracle.PartitionedStreamOracle(sizes, w.K, ff=0.9)
    U0 = so.modes.copy()
    off = 0
    for i, m in enumerate(sizes):
        po.U_all[off * w.K: (off + m) * w.K] = np.asfortranarray(U0[sum(sizes[:i]): sum(sizes[:i]) + m]).ravel(order="F")
        off += m
    po.s[:] = so.singular_values
    po.r = so.r
    for A in batches[1:]:
        so.incorporate(A)
        po.incorporate(_split_rows(A, sizes))
        assert po.r == so.r
        assert sigma_rel_err(po.singular_values, so.singular_values) <= 1e-12
        assert np.abs(po.modes - so.modes).max() <= 1e-10     # same sign rule on the same U~
        assert orth_err(po.modes) <= 1e-13


def test_pstream_partition_block_is_that_partitions_rows():
    # Each partition's modes are the rows of the stacked modes (a wrong block
    # index in the local lift would move rows between partitions).
    sig = np.linspace(2.0, 0.3, 6)
    A, _, _ = planted(400, 24, sig, seed=21)
    sizes = [100, 180, 120]
    po = oracle.PartitionedStreamOracle(sizes, 6, ff=1.0, r_local=8)
    po.incorporate(_split_rows(A[:, :12], sizes)).incorporate(_split_rows(A[:, 12:], sizes))
    Ul, sl, _ = np.linalg.svd(A, full_matrices=False)
    Us = align_signs(po.modes, Ul[:, :6])
    o = 0
    for i, m in enumerate(sizes):
        assert np.abs(align_signs(po.modes_part(i)[:, :6], Ul[o: o + m, :6]) - Us[o: o + m, :6]).max() <= 1e-10
        o += m


def test_pstream_exact_without_truncation():
    # Rank 6 = K, ff = 1, local truncation r_local >= local rank: the APMOS
    # initialisation and every partitioned update are exact, so the state is
    # the SVD of the concatenation of all batches (LAPACK).
    sig = np.linspace(3.0, 0.4, 6)
    A, _, _ = planted(700, 40, sig, seed=22)
    sizes = [150, 250, 300]
    po = oracle.PartitionedStreamOracle(sizes, 6, ff=1.0, r_local=10)
    for b in np.split(np.arange(40), 4):
        po.incorporate(_split_rows(A[:, b], sizes))
    Ul, sl, _ = np.linalg.svd(A, full_matrices=False)
    assert sigma_rel_err(po.singular_values[:6], sl[:6]) <= 1e-12
    assert max_principal_angle(po.modes[:, :6], Ul[:, :6]) <= 1e-10


def test_pstream_forget_factor_closed_form():
    # ff < 1 without truncation loss (rank 5 = K): batch j is weighted by ff^(last - j).
    ff = 0.85
    sig = np.linspace(2.5, 0.5, 5)
    A, _, _ = planted(360, 30, sig, seed=23)
    parts = [A[:, :10], A[:, 10:20], A[:, 20:]]
    sizes = [90, 130, 140]
    po = oracle.PartitionedStreamOracle(sizes, 5, ff=ff, r_local=10)
    for p in parts:
        po.incorporate(_split_rows(p, sizes))
    W = np.hstack([ff ** 2 * parts[0], ff * parts[1], parts[2]])
    Ul, sl, _ = np.linalg.svd(W, full_matrices=False)
    assert sigma_rel_err(po.singular_values[:5], sl[:5]) <= 1e-12
    assert max_principal_angle(po.modes[:, :5], Ul[:, :5]) <= 1e-10


def test_gradient_single_batch_closed_form():
    # One exact truncated SVD: L = ||A||^2 - sum s_j^2 + sum w_j s_j,
    # dL/dA = 2A - U_K (2 S_K - diag(w)) V_K^T.
    w = synth.scaled(synth.c5_gradient(), M=300, N=40, batches=1, K=5)
    A = np.asfortranarray(synth.numpy_cm(synth.planted_stream(w)[0]))
    wt = synth.loss_weights(w)
    G = oracle.stream_grad(A, w.K, 1.0, 1, wt)
    Ul, sl, Vt = np.linalg.svd(A, full_matrices=False)
    K = w.K
    ref = 2 * A - Ul[:, :K] @ np.diag(2 * sl[:K] - wt) @ Vt[:K]
    assert np.linalg.norm(G - ref) / np.linalg.norm(ref) <= 1e-10
    L, _, s = oracle.stream_loss(A, K, 1.0, 1, wt)
    assert abs(L - (np.sum(A * A) - np.sum(sl[:K] ** 2) + wt @ sl[:K])) <= 1e-11 * abs(L)


def test_gradient_stream_matches_finite_differences():
    # Streaming with truncation: reverse mode against central differences
    # along random directions (||D|| = ||A||, h = 1e-3 relative) and single coordinates.
    w = synth.scaled(synth.c5_gradient(), M=512, N=16, batches=4, K=6)
    A = np.hstack([synth.numpy_cm(t) for t in synth.planted_stream(w)])
    A = np.asfortranarray(A)
    wt = synth.loss_weights(w)
    G = oracle.stream_grad(A, w.K, 1.0, w.batches, wt)
    g = rng(77)
    h = 1e-3
    for t in range(8):
        D = g.standard_normal(A.shape)
        D *= np.linalg.norm(A) / np.linalg.norm(D)
        lp = oracle.stream_loss(A + h * D, w.K, 1.0, w.batches, wt)[0]
        lm = oracle.stream_loss(A - h * D, w.K, 1.0, w.batches, wt)[0]
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(G * D))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (t, fd, an)
    for t in range(8):
        i, j = int(g.integers(A.shape[0])), int(g.integers(A.shape[1]))
        hh = 1e-5
        Ap = A.copy(); Ap[i, j] += hh
        Am = A.copy(); Am[i, j] -= hh
        fd = (oracle.stream_loss(Ap, w.K, 1.0, w.batches, wt)[0] - oracle.stream_loss(Am, w.K, 1.0, w.batches, wt)[0]) / (2 * hh)
        assert abs(fd - G[i, j]) <= 1e-6 * max(1.0, np.abs(G).max()), (i, j, fd, G[i, j])


def test_gradient_stream_with_forget_factor():
    w = synth.scaled(synth.c5_gradient(), M=200, N=10, batches=3, K=4)
    A = np.asfortranarray(np.hstack([synth.numpy_cm(t) for t in synth.planted_stream(w)]))
    wt = synth.loss_weights(w)
    ff = 0.9
    G = oracle.stream_grad(A, w.K, ff, w.batches, wt)
    D = rng(5).standard_normal(A.shape)
    h = 1e-4
    fd = (oracle.stream_loss(A + h * D, w.K, ff, w.batches, wt)[0] - oracle.stream_loss(A - h * D, w.K, ff, w.batches, wt)[0]) / (2 * h)
    assert abs(fd - np.sum(G * D)) <= 1e-6 * max(1.0, abs(fd))


def test_matmul_nn_matches_blas():
    # the oracle's plain triple loop against LAPACK/BLAS-backed numpy (independent implementation)
    rng = np.random.default_rng(4)
    A = rng.standard_normal((37, 19))
    B = rng.standard_normal((19, 23))
    assert np.allclose(oracle.matmul_nn(A, B), A @ B, rtol=0, atol=1e-13)
    assert np.allclose(oracle.matmul_tn(A, rng.standard_normal((37, 5))).shape, (19, 5))


@pytest.mark.parametrize("k", [0, 300, 8193, 70000, 4_200_003])
def test_matmul_tn_chunked_reduction_exact(k):
    # Integer-valued operands keep every partial sum exact in FP64, so the
    # oracle's chunked reduction over the long dimension (chunks of 8192 rows,
    # widened beyond 512 chunks) must equal the integer product bit for bit:
    # a dropped, repeated or shifted chunk changes the result.
    rng = np.random.default_rng(11 + k % 97)
    m, n = (3, 2) if k > 100_000 else (19, 5)
    A = rng.integers(-8, 9, size=(k, m))
    B = rng.integers(-8, 9, size=(k, n))
    C = oracle.matmul_tn(A.astype(np.float64), B.astype(np.float64))
    ref = (A.T @ B).astype(np.float64)
    assert C.shape == (m, n)
    assert np.array_equal(C, ref)


def test_matmul_tn_against_blas_real_values():
    rng = np.random.default_rng(12)
    A = rng.standard_normal((70001, 7))
    B = rng.standard_normal((70001, 4))
    C = oracle.matmul_tn(A, B)
    bound = 70001 * 2.0 ** -52 * (np.abs(A).T @ np.abs(B))
    assert np.all(np.abs(C - A.T @ B) <= bound)


@pytest.mark.parametrize("m", [255, 256, 257, 600])
def test_matmul_nn_row_blocks_exact(m):
    # rows are split into blocks of 256: ragged and exact multiples, integer data (exact sums)
    rng = np.random.default_rng(13 + m)
    A = rng.integers(-8, 9, size=(m, 33))
    B = rng.integers(-8, 9, size=(33, 6))
    assert np.array_equal(oracle.matmul_nn(A.astype(np.float64), B.astype(np.float64)), (A @ B).astype(np.float64))


@pytest.mark.parametrize("m", [65536, 65537, 2 * 65536 + 5])
def test_hhqr_long_columns_chunked_norm(m):
    # The Householder vector norm is a sum of squares in chunks of 65536 entries.
    # Integer columns: the first column's squared norm is an exact integer, so
    # R_00 must be its correctly rounded square root; the rest is checked
    # against LAPACK after the sign normalisation (R_jj >= 0).
    rng = np.random.default_rng(14)
    A = rng.integers(-5, 6, size=(m, 3)).astype(np.float64)
    A[m - 1, 0] = 7.0   # an entry in the last (ragged) chunk
    Q, R = oracle.hhqr(A)
    exact = int(np.sum(A[:, 0].astype(np.int64) ** 2))
    assert R[0, 0] == np.sqrt(float(exact))
    Ql, Rl = np.linalg.qr(A)
    sg = np.sign(np.diag(Rl))
    Rl = sg[:, None] * Rl
    assert np.max(np.abs(R - Rl)) <= 1e-12 * np.abs(Rl).max()
    assert np.linalg.norm(Q.T @ Q - np.eye(3)) <= 1e-13
