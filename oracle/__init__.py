"""FP64 CPU oracle for the streaming / randomized / partitioned SVD (arXiv 2108.08845).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the product library never does, and
the two share no code.  The arithmetic lives in `psvd_oracle.c` (plain C,
FP64, no BLAS/LAPACK); this module only marshals numpy arrays.

Matrices are numpy float64 arrays of shape (rows, cols) in Fortran
(column-major) order, so each column (snapshot) is contiguous.

Functions and the passages they follow:
  philox4x32_10, omega  -- Gaussian test matrix (Sec. 3.3, drawn afresh for
                            every randomized SVD); Philox4x32-10 + Box-Muller.
  hhqr                  -- Householder thin QR, R_jj >= 0 (the QR of Algorithm 1).
  jacobi_svd            -- one-sided Jacobi SVD (the SVD of R in Algorithm 1; Eq. (9)).
  StreamOracle          -- Algorithm 1 per batch, deterministic or randomized
                            (Eqs. (7)-(11), Halko-Martinsson-Tropp power iterations).
  apmos                 -- Algorithm 2 / Eqs. (3)-(6); with `omega` the global
                            SVD of W is the low-rank SVD (the paper's placement).
  low_rank_svd          -- Eqs. (7)-(11) on a small matrix with a given test matrix.
  PartitionedStreamOracle -- the parallel streaming of Sec. 3 over row
                            partitions: APMOS initialisation, then per batch
                            local QR of each partition's panel, QR of the
                            stacked R factors, SVD of the combined R, local lift.
  stream_loss, stream_grad -- loss ||A - U U^T A||^2 + sum w_j s_j of the
                            streamed truncated SVD and its reverse-mode gradient.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpsvd_oracle.so")
_lib = None

OK = 0
EINVAL = -1
ENOMEM = -4
ENOCONV = -6

PREC_F64, PREC_F32, PREC_BF16 = 0, 1, 2

_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
    lib.orc_philox4x32_10.restype = None
    lib.orc_omega.argtypes = [ctypes.c_uint64, _i64, _i64, _i64, ctypes.c_int, _dp]
    lib.orc_omega.restype = None
    lib.orc_hhqr.argtypes = [_i64, _i64, _dp, _i64, _dp, _dp]
    lib.orc_jacobi_svd.argtypes = [_i64, _i64, _dp, _i64, _dp, _dp, _dp, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int)]
    lib.orc_stream_update.argtypes = [_i64, _i32, ctypes.c_double, _i32, _i32, _dp, _i64, _dp,
                                      ctypes.POINTER(_i32), _dp, _i64, _i64, _dp, _dp]
    lib.orc_apmos.argtypes = [_i32, ctypes.POINTER(_i64), _i64, _i32, _i32, _dp, _dp, _dp, _dp]
    lib.orc_pstream_update.argtypes = [_i32, ctypes.POINTER(_i64), _i32, ctypes.c_double, _dp, _dp,
                                       ctypes.POINTER(_i32), _dp, _i64]
    lib.orc_stream_loss.argtypes = [_i64, _i32, ctypes.c_double, _i32, _i64, _dp, _i64, _dp, _dp, _dp, _dp]
    lib.orc_stream_grad.argtypes = [_i64, _i32, ctypes.c_double, _i32, _i64, _dp, _i64, _dp, _dp]
    lib.orc_low_rank_svd.argtypes = [_i64, _i64, _dp, _i64, _i32, _dp, _i64, _dp, _i64, _dp, ctypes.POINTER(_i32)]
    lib.orc_apmos_lr.argtypes = [_i32, ctypes.POINTER(_i64), _i64, _i32, _i32, _dp, _dp, _i64, _dp, _dp, _dp]
    lib.orc_pstream_update_lr.argtypes = [_i32, ctypes.POINTER(_i64), _i32, ctypes.c_double, _dp, _dp,
                                          ctypes.POINTER(_i32), _dp, _i64, _dp, _i64]
    lib.orc_matmul_nn.argtypes = [_i64, _i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64]
    lib.orc_matmul_nn.restype = None
    lib.orc_matmul_tn.argtypes = [_i64, _i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64]
    lib.orc_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a):
    return np.asfortranarray(a, dtype=np.float64)


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _check(rc, what):
    if rc != OK:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def num_threads() -> int:
    return _load().orc_num_threads()


def philox4x32_10(ctr, key):
    """Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib.orc_philox4x32_10(c, k, o)
    return [int(o[i]) for i in range(4)]


def omega(seed: int, batch: int, n: int, ell: int, precision: int) -> np.ndarray:
    """Gaussian test matrix (n x ell, column-major) for one batch, rounded to the path's precision."""
    out = np.zeros((n, ell), dtype=np.float64, order="F")
    _load().orc_omega(ctypes.c_uint64(seed), batch, n, ell, precision, _ptr(out))
    return out


def hhqr(A):
    A = _f64(A)
    m, n = A.shape
    Q = np.zeros((m, n), order="F")
    R = np.zeros((n, n), order="F")
    _check(_load().orc_hhqr(m, n, _ptr(A), max(m, 1), _ptr(Q), _ptr(R)), "hhqr")
    return Q, R


def jacobi_svd(A, max_sweeps: int = 60):
    """A = U diag(s) V^T for a tall (m >= n) A; s descending."""
    A = _f64(A)
    m, n = A.shape
    U = np.zeros((m, n), order="F")
    s = np.zeros(n)
    V = np.zeros((n, n), order="F")
    sw = ctypes.c_int(0)
    rc = _load().orc_jacobi_svd(m, n, _ptr(A), max(m, 1), _ptr(U), _ptr(s), _ptr(V), max_sweeps, ctypes.byref(sw))
    _check(rc, "jacobi_svd")
    return U, s, V


def matmul_tn(A, B):
    """A^T B with a fixed-order reduction (A: k x m, B: k x n)."""
    A = _f64(A)
    B = _f64(B)
    k, m = A.shape
    n = B.shape[1]
    C = np.zeros((m, n), order="F")
    _check(_load().orc_matmul_tn(m, n, k, _ptr(A), max(k, 1), _ptr(B), max(k, 1), _ptr(C), max(m, 1)), "matmul_tn")
    return C


def matmul_nn(A, B):
    """A B with a fixed-order reduction (A: m x k, B: k x n)."""
    A = _f64(A)
    B = _f64(B)
    m, k = A.shape
    n = B.shape[1]
    C = np.zeros((m, n), order="F")
    _load().orc_matmul_nn(m, n, k, _ptr(A), max(m, 1), _ptr(B), max(k, 1), _ptr(C), max(m, 1))
    return C


class StreamOracle:
    """Algorithm 1, one `incorporate(A)` per batch.

    `ell = K + oversampling`; when `ell == 0` (deterministic mode) or
    `ell >= r + N` the deterministic step runs, otherwise the randomized
    range finder with the batch's Gaussian test matrix `omega(seed, batch,
    r + N, ell, precision)`.  `omega_precision` selects how the test matrix
    is rounded (PREC_F64 / PREC_F32 / PREC_BF16), matching the path compared.
    """

    def __init__(self, M, K, ff=1.0, oversampling=0, power_iters=0, randomized=False, seed=0,
                 omega_precision=PREC_F64):
        self.M, self.K, self.ff = int(M), int(K), float(ff)
        self.ell = int(K + oversampling) if randomized else 0
        self.q = int(power_iters)
        self.seed = int(seed)
        self.omega_precision = omega_precision
        self.U = np.zeros((self.M, self.K), order="F")
        self.s = np.zeros(self.K)
        self.r = 0
        self.batch = 0
        self.last_small_u = None

    def incorporate(self, A, omega_override=None):
        A = _f64(A)
        M, N = A.shape
        assert M == self.M
        if N == 0:
            return self
        n = self.r + N
        Om = None
        if self.ell > 0 and self.ell < n:
            Om = omega_override if omega_override is not None else omega(
                self.seed, self.batch, n, self.ell, self.omega_precision)
            Om = _f64(Om)
        rk_cap = min(self.K, self.ell if Om is not None else n)
        small = np.zeros(((self.ell if Om is not None else n), rk_cap), order="F")
        r = _i32(self.r)
        rc = _load().orc_stream_update(self.M, self.K, self.ff, self.ell, self.q, _ptr(self.U), self.M,
                                       _ptr(self.s), ctypes.byref(r), _ptr(A), N, max(M, 1), _ptr(Om),
                                       _ptr(small))
        _check(rc, "stream_update")
        self.r = int(r.value)
        self.batch += 1
        self.last_small_u = small
        return self

    initialize = incorporate

    @property
    def modes(self):
        return self.U[:, : self.r]

    @property
    def singular_values(self):
        return self.s[: self.r].copy()


def low_rank_svd(A, K, Om):
    """Low-rank SVD of a small matrix A (m x n) with test matrix Om (n x ell):
    Eqs. (7)-(11) without power iterations -> (U (m x k), s (k)), k = min(K, ell)."""
    A = _f64(A)
    Om = _f64(Om)
    m, n = A.shape
    ell = Om.shape[1]
    k = min(int(K), ell)
    U = np.zeros((m, k), order="F")
    s = np.zeros(max(k, 1))
    kk = _i32(0)
    rc = _load().orc_low_rank_svd(m, n, _ptr(A), m, int(K), _ptr(Om), ell, _ptr(U), m, _ptr(s), ctypes.byref(kk))
    _check(rc, "low_rank_svd")
    return U[:, : kk.value], s[: kk.value].copy()


def apmos(parts, r, K, omega=None):
    """Algorithm 2 on a list of (M_i x N) partitions -> (list of U^i, Lambda~ (K), X~ (N x K)).
    With `omega` (P r x ell) the SVD of W is the low-rank SVD of Eqs. (7)-(11)."""
    parts = [_f64(p) for p in parts]
    P = len(parts)
    N = parts[0].shape[1]
    Ms = np.array([p.shape[0] for p in parts], dtype=np.int64)
    A_all = np.concatenate([p.ravel(order="F") for p in parts])
    U_all = np.zeros(int(Ms.sum()) * K)
    Lam = np.zeros(K)
    X = np.zeros((N, K), order="F")
    if omega is None:
        rc = _load().orc_apmos(P, Ms.ctypes.data_as(ctypes.POINTER(_i64)), N, r, K, _ptr(A_all), _ptr(U_all),
                               _ptr(Lam), _ptr(X))
    else:
        Om = _f64(omega)
        assert Om.shape[0] == P * r
        rc = _load().orc_apmos_lr(P, Ms.ctypes.data_as(ctypes.POINTER(_i64)), N, r, K, _ptr(A_all), _ptr(Om),
                                  Om.shape[1], _ptr(U_all), _ptr(Lam), _ptr(X))
    _check(rc, "apmos")
    out, off = [], 0
    for m in Ms:
        out.append(U_all[off: off + m * K].reshape((m, K), order="F"))
        off += m * K
    return out, Lam, X


class PartitionedStreamOracle:
    """The parallel streaming SVD of Sec. 3 on P row partitions (M_i rows each).

    The first batch initialises the state with APMOS (Algorithm 2 with local
    truncation `r_local`, K global modes); every later batch runs the
    partitioned update `orc_pstream_update` (local QR per partition, QR of
    the stacked R factors, SVD of the combined R, U^i = Q^i Q_g^i U~_K).
    `modes` is the stacked U (sum M_i x r), `modes_part(i)` one partition's.
    """

    def __init__(self, M_parts, K, ff=1.0, r_local=None, low_rank=False, seed=0, omega_precision=PREC_F64):
        self.Ms = np.array([int(m) for m in M_parts], dtype=np.int64)
        self.P, self.K, self.ff = len(self.Ms), int(K), float(ff)
        self.r_local = r_local
        self.U_all = np.zeros(int(self.Ms.sum()) * self.K)
        self.s = np.zeros(self.K)
        self.r = 0
        # the paper's placement of randomization: the SVD of W (initialisation)
        # and of the combined R factor (updates) by the low-rank SVD with a
        # K-column test matrix, drawn for update b from (seed, b)
        self.low_rank, self.seed, self.omega_precision = bool(low_rank), int(seed), int(omega_precision)
        self.batch = 0

    def _stack(self, parts):
        parts = [_f64(p) for p in parts]
        assert len(parts) == self.P and all(p.shape[0] == m for p, m in zip(parts, self.Ms))
        return parts, np.concatenate([p.ravel(order="F") for p in parts])

    def incorporate(self, parts):
        parts, A_all = self._stack(parts)
        N = parts[0].shape[1]
        if N == 0:
            return self
        if self.r == 0:
            rl = int(self.r_local) if self.r_local is not None else min(self.K, N)
            om = omega(self.seed, self.batch, self.P * rl, self.K, self.omega_precision) if self.low_rank else None
            Us, lam, _ = apmos(parts, rl, self.K, omega=om)
            off = 0
            for u, m in zip(Us, self.Ms):
                self.U_all[off: off + m * self.K] = u.ravel(order="F")
                off += m * self.K
            self.s[:] = lam
            self.r = self.K
            self.batch += 1
            return self
        r = _i32(self.r)
        if self.low_rank:
            n = self.r + N
            om = omega(self.seed, self.batch, n, min(self.K, n), self.omega_precision)
            rc = _load().orc_pstream_update_lr(self.P, self.Ms.ctypes.data_as(ctypes.POINTER(_i64)), self.K, self.ff,
                                               _ptr(self.U_all), _ptr(self.s), ctypes.byref(r), _ptr(A_all), N,
                                               _ptr(om), om.shape[1])
        else:
            rc = _load().orc_pstream_update(self.P, self.Ms.ctypes.data_as(ctypes.POINTER(_i64)), self.K, self.ff,
                                            _ptr(self.U_all), _ptr(self.s), ctypes.byref(r), _ptr(A_all), N)
        _check(rc, "pstream_update")
        self.r = int(r.value)
        self.batch += 1
        return self

    initialize = incorporate

    def modes_part(self, i):
        off = int(self.Ms[:i].sum()) * self.K
        m = int(self.Ms[i])
        return self.U_all[off: off + m * self.K].reshape((m, self.K), order="F")[:, : self.r]

    @property
    def modes(self):
        return np.vstack([self.modes_part(i) for i in range(self.P)])

    @property
    def singular_values(self):
        return self.s[: self.r].copy()


def stream_loss(A, K, ff, batches, w):
    """Loss of the deterministic stream over `batches` equal column batches of A; returns (L, U, s)."""
    A = _f64(A)
    M, Nt = A.shape
    assert Nt % batches == 0
    w = np.ascontiguousarray(w, dtype=np.float64)
    L = ctypes.c_double(0.0)
    U = np.zeros((M, K), order="F")
    s = np.zeros(K)
    rc = _load().orc_stream_loss(M, K, ff, batches, Nt // batches, _ptr(A), M, _ptr(w), ctypes.byref(L),
                                 _ptr(U), _ptr(s))
    _check(rc, "stream_loss")
    return L.value, U, s


def stream_grad(A, K, ff, batches, w):
    """Reverse-mode dL/dA of `stream_loss`."""
    A = _f64(A)
    M, Nt = A.shape
    w = np.ascontiguousarray(w, dtype=np.float64)
    G = np.zeros((M, Nt), order="F")
    rc = _load().orc_stream_grad(M, K, ff, batches, Nt // batches, _ptr(A), M, _ptr(w), _ptr(G))
    _check(rc, "stream_grad")
    return G
