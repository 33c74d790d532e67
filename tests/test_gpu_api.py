"""GPU tests of the one-shot randomized SVD and of state checkpoints.

psvd_rsvd (Sec. 3.3, Eqs. (7)-(11)) is one randomized update of an empty
stream: its U and sigma are compared with the FP64 oracle's randomized step
on the same Gaussian test matrix, and V with its defining relation
A^T U = V S (Eq. (11): B = Q^T A = U~ S V~^T, U = Q U~).  Checkpoints:
a stream saved after some batches and resumed in a fresh handle reproduces
the uninterrupted stream bit for bit (the test matrix of each update is a
function of the seed and the batch count).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from conftest import sigma_rel_err, max_principal_angle, orth_err

pytestmark = pytest.mark.gpu


def lib():
    import paper_2108_08845_amd as P
    return P


def planted(M, N, rank, seed, dtype=torch.float64, decay=0.7):
    g = torch.Generator().manual_seed(seed)
    U, _ = torch.linalg.qr(torch.randn(M, rank, generator=g, dtype=torch.float64))
    V, _ = torch.linalg.qr(torch.randn(N, rank, generator=g, dtype=torch.float64))
    s = decay ** torch.arange(rank, dtype=torch.float64)
    A = (U * s) @ V.T + 1e-8 * torch.randn(M, N, generator=g, dtype=torch.float64)
    return A.to(dtype)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_rsvd_matches_oracle(precision, tol):
    M, N, K, p, q, seed = 3000, 200, 12, 8, 2, 7
    dt = torch.float64 if precision == "fp64" else torch.float32
    A = planted(M, N, 60, 11, dt)
    P = lib()
    Ag = A.cuda()
    U, s, V = P.rsvd(Ag, K, oversampling=p, power_iters=q, seed=seed, precision=precision)
    U = U.double().cpu().numpy()
    V = V.double().cpu().numpy()
    so = oracle.StreamOracle(M, K, oversampling=p, power_iters=q, randomized=True, seed=seed,
                             omega_precision=oracle.PREC_F64 if precision == "fp64" else oracle.PREC_F32)
    An = np.asfortranarray(A.double().numpy())
    so.incorporate(An)
    assert len(s) == K
    assert sigma_rel_err(s, so.singular_values) <= tol
    assert max_principal_angle(U[:, :8], so.modes[:, :8]) <= 100 * tol
    assert orth_err(U) <= (1e-12 if precision == "fp64" else 1e-5)
    # Eq. (11): A^T U = V S, and V has orthonormal columns
    resid = np.linalg.norm(An.T @ U - V * s) / np.linalg.norm(V * s)
    assert resid <= 10 * tol
    assert orth_err(V) <= 1e2 * tol


def test_rsvd_exact_when_sketch_covers_rank():
    # rank 10 <= K + p: the randomized range finder is exact (HMT Thm. 1.1).
    # The sketch Gram Y^T Y then has rank 10 < K + p; its Cholesky factor
    # would carry errors of order one, so the small core takes the eigen
    # route (orthonormal basis of the numerical range of Y) and the result is
    # exact to rounding.
    M, N = 2048, 96
    g = torch.Generator().manual_seed(3)
    U0, _ = torch.linalg.qr(torch.randn(M, 10, generator=g, dtype=torch.float64))
    V0, _ = torch.linalg.qr(torch.randn(N, 10, generator=g, dtype=torch.float64))
    s0 = torch.linspace(5.0, 1.0, 10, dtype=torch.float64)
    A = (U0 * s0) @ V0.T
    U, s, V = lib().rsvd(A.cuda(), 10, oversampling=6, power_iters=0, seed=1, precision="fp64")
    assert np.max(np.abs(s - s0.numpy()) / s0.numpy()) <= 1e-12
    R = (U.cpu() * torch.as_tensor(s)) @ V.cpu().T
    assert float((R - A).norm() / A.norm()) <= 1e-12
    assert orth_err(U.cpu().numpy()) <= 1e-12


def test_rsvd_rejects_bad_arguments():
    P = lib()
    A = torch.zeros(100, 20, dtype=torch.float32, device="cuda")
    with pytest.raises(P.PsvdError):
        P.rsvd(A, 0)
    with pytest.raises(P.PsvdError):
        P.rsvd(A, 21)
    with pytest.raises(P.PsvdError):          # FP64 data needs the FP64 precision
        P.rsvd(A.double(), 5, precision="fp32")


@pytest.mark.parametrize("precision,randomized", [("fp32", True), ("mixed", True), ("fp64", False)])
def test_checkpoint_resume_is_bitwise(precision, randomized):
    w = synth.scaled(synth.c2_randomized_fp32(), M=1 << 13, N=48, batches=5, K=12)
    dt = torch.float64 if precision == "fp64" else torch.float32
    bs = [b.to(dt).cuda() for b in synth.planted_stream(w)]
    P = lib()
    kw = dict(ff=w.ff, oversampling=6, power_iters=1, randomized=randomized, precision=precision, seed=9)
    a = P.StreamingSVD(w.M, w.K, **kw)
    for b in bs:
        a.incorporate_data(b.t())
    b1 = P.StreamingSVD(w.M, w.K, **kw)
    for b in bs[:2]:
        b1.incorporate_data(b.t())
    state = b1.save_state()
    b1.close()
    c = P.StreamingSVD(w.M, w.K, **kw)
    c.load_state(state)
    assert c.rank == min(w.K, 2 * w.N)
    for b in bs[2:]:
        c.incorporate_data(b.t())
    assert np.array_equal(a.singular_values, c.singular_values)
    assert torch.equal(a.modes, c.modes)
    # a different configuration is refused and leaves the handle untouched
    d = P.StreamingSVD(w.M, w.K, **dict(kw, seed=10))
    with pytest.raises(P.PsvdError):
        d.load_state(state)
    assert d.rank == 0
    with pytest.raises(P.PsvdError):
        c.load_state(state[:100])
    assert np.array_equal(a.singular_values, c.singular_values)


@pytest.mark.parametrize("precision,async_updates", [("mixed", True), ("fp32", False), ("fp64", True)])
def test_graph_updates_match_eager_launches(precision, async_updates):
    """A randomized update run as one captured hipGraph (graph=True: updated in
    place when only the batch and the state buffers change) and the same updates
    launched one by one give bit-identical modes and singular values after every
    update, with eager work and synchronisation of the program between the
    replays."""
    w = synth.scaled(synth.c2_randomized_fp32(), M=1 << 13, N=48, batches=6, K=12)
    dt = torch.float64 if precision == "fp64" else torch.float32
    bs = [b.to(dt).cuda() for b in synth.planted_stream(w)]
    P = lib()
    kw = dict(ff=w.ff, oversampling=6, power_iters=2, randomized=True, precision=precision, seed=5,
              async_updates=async_updates)
    g = P.StreamingSVD(w.M, w.K, graph=True, **kw)
    e = P.StreamingSVD(w.M, w.K, graph=False, **kw)
    for b in bs + bs[:2]:
        g.incorporate_data(b.t())
        scratch = (b.double() * 2.0).sum()   # eager work between the replays
        e.incorporate_data(b.t())
        torch.cuda.synchronize()
        assert torch.isfinite(scratch)
        assert np.array_equal(g.singular_values, e.singular_values)
        assert torch.equal(g.modes, e.modes)


def test_async_device_error_surfaces_at_next_sync():
    # With asynchronous updates a device-side failure (here NaN data reaching
    # the small factorisation) is reported by the next synchronising call.
    P = lib()
    M, N = 4096, 32
    g = torch.Generator(device="cuda").manual_seed(2)
    A = torch.randn(N, M, generator=g, device="cuda")
    svd = P.StreamingSVD(M, 8, oversampling=4, power_iters=1, randomized=True, precision="fp32",
                         async_updates=True)
    svd.incorporate_data(A.t())
    assert len(svd.singular_values) == 8          # clean so far
    bad = A.clone()
    bad[3, 17] = float("nan")
    svd.incorporate_data(bad.t())                 # returns before the device work ends
    with pytest.raises(P.PsvdError) as e:
        svd.singular_values
    assert e.value.code == -5                     # PSVD_E_NONFINITE
    st = svd.stats()                              # reported once, then cleared
    assert st["last_sweeps"] >= 0
