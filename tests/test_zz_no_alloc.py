"""The allocation-free one-shot randomized SVD (psvd_rsvd_noalloc) against psvd_rsvd.

Both entry points run the same kernels with the same launch shapes on the
same input and test matrix; only where the workspace lives differs (the
library's fixed device array instead of allocations), so the results must
agree bit for bit.  Two calls in a row, the second on a smaller problem,
check that nothing the first call left in the shared array leaks into the
second.  A problem larger than the fixed array is refused with a clear error.
"""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def lib():
    import paper_2108_08845_amd as P
    return P


def planted(M, N, rank, seed, dtype):
    g = torch.Generator().manual_seed(seed)
    U, _ = torch.linalg.qr(torch.randn(M, rank, generator=g, dtype=torch.float64))
    V, _ = torch.linalg.qr(torch.randn(N, rank, generator=g, dtype=torch.float64))
    s = 0.8 ** torch.arange(rank, dtype=torch.float64)
    A = (U * s) @ V.T + 1e-6 * torch.randn(M, N, generator=g, dtype=torch.float64)
    return A.to(dtype)


# (M, N, K, p, q, seed): a randomized case, then a smaller ragged one; the last
# precision row (p + K >= N) takes the exact deterministic step.
CASES = {
    "mixed": [(40000, 200, 20, 10, 2, 5), (30001, 64, 10, 6, 1, 6)],
    "fp32": [(40000, 200, 20, 10, 2, 5), (30001, 64, 10, 6, 1, 6)],
    "fp64": [(20000, 96, 12, 8, 1, 7), (5000, 20, 10, 12, 0, 8)],
}


@pytest.mark.parametrize("precision", ["mixed", "fp32", "fp64"])
def test_noalloc_matches_rsvd_two_calls(precision):
    P = lib()
    dt = torch.float64 if precision == "fp64" else torch.float32
    for (M, N, K, p, q, seed) in CASES[precision]:
        print(f"noalloc {precision} M={M} N={N} K={K} p={p} q={q}", flush=True)
        A = planted(M, N, min(40, N), seed, dt).cuda()
        U0, s0, V0 = P.rsvd(A, K, oversampling=p, power_iters=q, seed=seed, precision=precision)
        U1, s1, V1 = P.rsvd_noalloc(A, K, oversampling=p, power_iters=q, seed=seed, precision=precision)
        torch.cuda.synchronize()
        assert len(s1) == len(s0) == min(K, N)
        assert np.array_equal(s0, s1)
        assert torch.equal(U0, U1)
        assert torch.equal(V0, V1)


def test_noalloc_refuses_beyond_the_fixed_array():
    P = lib()
    M, N, K = 1 << 22, 64, 40          # kept sketch alone: 2^22 x 50 x 4 B > 256 MiB
    A = torch.empty((N, M), dtype=torch.float32, device="cuda").t()
    with pytest.raises(P.PsvdError) as ei:
        P.rsvd_noalloc(A, K, oversampling=10, power_iters=0, precision="fp32")
    assert ei.value.code == -4
    assert "fixed maximum" in str(ei.value)


def test_noalloc_rejects_mismatched_output_type():
    P = lib()
    L = P._lib.load()
    M, N = 1000, 30
    A = torch.zeros((N, M), dtype=torch.float32, device="cuda")
    U = torch.zeros((5, M), dtype=torch.float64, device="cuda")
    s = np.zeros(5)
    rank = ctypes.c_int32()
    rc = L.psvd_rsvd_noalloc(ctypes.c_void_p(A.data_ptr()), M, N, M, P._lib.PSVD_F32, 5, 2, 0, ctypes.c_uint64(0),
                             P._lib.PREC_FP32, ctypes.c_void_p(U.data_ptr()), M, None, N, P._lib.PSVD_F64,
                             s.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(rank), None)
    assert rc == -3
