"""MI355X streaming / randomized / partitioned SVD (after arXiv 2108.08845, "PyParSVD").

Python surface over the C ABI of include/psvd.h.  Matrices follow the paper's
orientation -- a batch A is M x N (rows are grid points, columns snapshots) --
stored column-major on the GPU: pass `X.T` for a contiguous torch tensor X of
shape (N, M).  PyTorch only provides device memory and the stream.

    svd = StreamingSVD(M, K, ff=0.95, oversampling=10, power_iters=2,
                       randomized=True, precision="mixed", seed=1)
    svd.initialize(A0)             # Algorithm 1, initialisation
    svd.incorporate_data(A1)       # Algorithm 1, per-batch update
    U, s = svd.modes, svd.singular_values
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import PsvdError

__all__ = ["StreamingSVD", "PartitionedStreamingSVD", "apmos_batched", "PsvdError", "stream_backward", "loss_and_grad", "StreamingSVDFunction",
           "rsvd", "rsvd_noalloc"]

_PREC = {"fp64": _lib.PREC_FP64, "fp32": _lib.PREC_FP32, "mixed": _lib.PREC_MIXED, "bf16": _lib.PREC_BF16}


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _as_colmajor(A):
    """(M, N) CUDA tensor -> (pointer, M, N, lda, dtype code, keep-alive tensor), column-major."""
    if not isinstance(A, torch.Tensor) or not A.is_cuda:
        raise TypeError("expected a CUDA tensor of shape (M, N)")
    if A.dim() != 2:
        raise ValueError("expected a 2-D (M, N) tensor")
    if A.dtype not in (torch.float32, torch.float64):
        raise TypeError("dtype must be float32 or float64")
    M, N = A.shape
    if not (A.stride(0) == 1 and (N <= 1 or A.stride(1) >= M)):
        A = A.t().contiguous().t()          # layout copy only
    lda = max(A.stride(1) if N > 1 else M, M)
    code = _lib.PSVD_F64 if A.dtype == torch.float64 else _lib.PSVD_F32
    return ctypes.c_void_p(A.data_ptr()), M, N, lda, code, A


class StreamingSVD:
    """Streaming truncated SVD of Algorithm 1 on one GPU (handle of the C library).

    ff: forget factor in (0, 1].  randomized: use the randomized range finder
    (sketch width K + oversampling, `power_iters` power iterations) whenever it
    is narrower than the panel.  precision: "fp64", "fp32", "mixed" (FP32 power
    passes, split-BF16 final projection) or "bf16" (BF16 power passes, the
    unrefined sketch).
    """

    def __init__(self, M, K, ff=1.0, oversampling=0, power_iters=0, randomized=False, precision="fp64",
                 seed=0, stream=None, async_updates=False, max_sweeps=60, fallback=True, profile=False,
                 tile_rows=0, wg_per_cu=0, omega_bf16=False, panel_width=0, split_m=0, autotuned=True, graph=False):
        self._libh = _lib.load()
        opt = _lib.Options()
        self._libh.psvd_default_options(ctypes.byref(opt))
        opt.method = _lib.RANDOMIZED if randomized else _lib.DETERMINISTIC
        opt.precision = _PREC[precision]
        opt.seed = int(seed)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        opt.stream = _stream_ptr(self._stream).value
        opt.max_sweeps = int(max_sweeps)
        opt.tile_rows = int(tile_rows)
        opt.wg_per_cu = int(wg_per_cu)
        opt.panel_width = int(panel_width)
        opt.split_m = int(split_m)
        opt.flags = ((_lib.OPT_ASYNC if async_updates else 0) | (0 if fallback else _lib.OPT_NO_FALLBACK)
                     | (_lib.OPT_PROFILE if profile else 0) | (_lib.OPT_OMEGA_BF16 if omega_bf16 else 0)
                     | (_lib.OPT_GRAPH if graph else 0))
        h = ctypes.c_void_p()
        rc = self._libh.psvd_initialize(ctypes.byref(h), int(M), int(K), float(ff), int(oversampling),
                                        int(power_iters), ctypes.byref(opt))
        _lib.check(rc, None, "psvd_initialize")
        self._h = h
        self.M, self.K, self.ff = int(M), int(K), float(ff)
        # launch parameters from the autotuner's cache, applied once the batch
        # width is known, unless the caller set any of them
        self._tune_pending = bool(autotuned) and not (tile_rows or wg_per_cu or panel_width or split_m)
        self.tuning = None
        self._tune_key = (int(oversampling), int(power_iters), precision, bool(randomized))
        self.oversampling, self.power_iters = int(oversampling), int(power_iters)
        self.randomized, self.precision, self.seed = bool(randomized), precision, int(seed)
        self._keep = None

    def close(self):
        if getattr(self, "_h", None):
            self._libh.psvd_finalize(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply_tuning(self, tile_rows=0, wg_per_cu=0, panel_width=0, split_m=0):
        """Set the launch parameters of the tall-panel kernels (psvd_set_tuning)."""
        rc = self._libh.psvd_set_tuning(self._h, int(tile_rows), int(wg_per_cu), int(panel_width), int(split_m))
        _lib.check(rc, self._h, "set_tuning")

    def _apply_cached_tuning(self, N):
        self._tune_pending = False
        p, q, precision, randomized = self._tune_key
        if not randomized:
            return
        from . import autotune
        opts = autotune.cached_options(self.M, N, self.K, p, q, precision)
        if opts is not None:
            self.apply_tuning(**opts)
            self.tuning = opts

    def incorporate_data(self, A):
        """Ingest one batch A (M x N CUDA tensor, column-major preferred)."""
        ptr, M, N, lda, code, keep = _as_colmajor(A)
        if self._tune_pending:
            self._apply_cached_tuning(N)
        self._keep = keep   # the update reads A on the stream
        rc = self._libh.psvd_incorporate_data(self._h, ptr, M, N, lda, code)
        _lib.check(rc, self._h, "incorporate_data")
        return self

    def initialize(self, A):
        """First batch (the initialisation of Algorithm 1); same as incorporate_data on an empty state."""
        if self.rank != 0:
            raise PsvdError(-9, "initialize() on a non-empty state")
        return self.incorporate_data(A)

    @property
    def rank(self):
        r = ctypes.c_int32()
        _lib.check(self._libh.psvd_rank(self._h, ctypes.byref(r)), self._h)
        return int(r.value)

    @property
    def singular_values(self):
        r = self.rank
        out = np.zeros(max(r, 1), dtype=np.float64)
        rr = ctypes.c_int32()
        rc = self._libh.psvd_singular_values(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             out.size, ctypes.byref(rr))
        _lib.check(rc, self._h, "singular_values")
        return out[:rr.value].copy()

    def modes_as(self, dtype=None):
        r = self.rank
        dt = dtype or (torch.float64 if self.precision == "fp64" else torch.float32)
        out = torch.empty((r, self.M), dtype=dt, device="cuda")
        if r:
            code = _lib.PSVD_F64 if dt == torch.float64 else _lib.PSVD_F32
            rc = self._libh.psvd_modes(self._h, ctypes.c_void_p(out.data_ptr()), self.M, code)
            _lib.check(rc, self._h, "modes")
        return out.t()

    @property
    def modes(self):
        """M x r modes (column-major CUDA tensor, a copy)."""
        return self.modes_as()

    def omega(self, batch, n):
        """The Gaussian test matrix of update `batch` on an n-column panel (numpy, n x (K + p))."""
        ell = self.K + self.oversampling
        out = np.zeros((ell, n), dtype=np.float64)   # column-major n x ell
        rc = self._libh.psvd_get_omega(self._h, int(batch), int(n), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        _lib.check(rc, self._h, "get_omega")
        return out.T

    def stats(self):
        s = _lib.Stats()
        _lib.check(self._libh.psvd_stats(self._h, ctypes.byref(s)), self._h)
        out = {k: getattr(s, k) for k, _ in _lib.Stats._fields_[:5]}
        out["kernels"] = {name: {"launches": int(s.kernel_launches[i]), "ms": float(s.kernel_ms[i])}
                          for i, name in enumerate(_lib.KERNEL_CLASSES)}
        return out

    def reset_stats(self):
        _lib.check(self._libh.psvd_reset_stats(self._h), self._h)

    @property
    def last_error(self):
        return self._libh.psvd_last_error(self._h).decode()

    def save_state(self):
        """Checkpoint (bytes) of U, s, the rank and the batch count; see load_state."""
        size = ctypes.c_size_t()
        _lib.check(self._libh.psvd_save_state(self._h, None, 0, ctypes.byref(size)), self._h, "save_state")
        buf = ctypes.create_string_buffer(size.value)
        _lib.check(self._libh.psvd_save_state(self._h, buf, size.value, ctypes.byref(size)), self._h, "save_state")
        return buf.raw

    def load_state(self, state):
        """Restore a checkpoint taken from a stream with the same configuration."""
        buf = ctypes.create_string_buffer(bytes(state), len(state))
        _lib.check(self._libh.psvd_load_state(self._h, buf, len(state)), self._h, "load_state")
        return self


class PartitionedStreamingSVD:
    """Partitioned streaming SVD (the parallel variant of Sec. 3) over row partitions on one GPU.

    M_parts: rows of each partition.  The first batch initialises the modes by
    APMOS (local truncation `r_local`, 0 = min(K, N)); later batches combine the
    partitions' QR factors.  precision "fp64" (FP64 data) or "fp32" (FP32 data).
    low_rank: the paper's placement of randomization -- the SVD of W and of the
    combined R factor by the low-rank SVD with a K-column test matrix (seed).
    """

    def __init__(self, M_parts, K, ff=1.0, r_local=0, precision="fp64", stream=None, max_sweeps=60, profile=False,
                 low_rank=False, seed=0):
        self._libh = _lib.load()
        opt = _lib.Options()
        self._libh.psvd_default_options(ctypes.byref(opt))
        opt.method = _lib.RANDOMIZED if low_rank else _lib.DETERMINISTIC
        opt.seed = int(seed)
        opt.precision = _PREC[precision]
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        opt.stream = _stream_ptr(self._stream).value
        opt.max_sweeps = int(max_sweeps)
        opt.flags = _lib.OPT_PROFILE if profile else 0
        self.M_parts = [int(m) for m in M_parts]
        P = len(self.M_parts)
        Ms = (ctypes.c_int64 * P)(*self.M_parts)
        h = ctypes.c_void_p()
        rc = self._libh.psvd_pstream_initialize(ctypes.byref(h), P, Ms, int(K), float(ff), int(r_local),
                                                ctypes.byref(opt))
        _lib.check(rc, None, "psvd_pstream_initialize")
        self._h = h
        self.K, self.ff, self.precision = int(K), float(ff), precision
        self._keep = None

    def close(self):
        if getattr(self, "_h", None):
            self._libh.psvd_finalize(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def incorporate_data(self, parts):
        """Ingest one batch given as its row partitions (list of M_i x N CUDA tensors)."""
        P = len(self.M_parts)
        if len(parts) != P:
            raise ValueError("one tensor per partition")
        cols = [_as_colmajor(p) for p in parts]
        for c, m in zip(cols, self.M_parts):
            if c[1] != m:
                raise ValueError("partition row count differs from M_parts")
        N = cols[0][2]
        self._keep = [c[5] for c in cols]
        A_ptrs = (ctypes.c_void_p * P)(*[c[0].value for c in cols])
        lds = (ctypes.c_int64 * P)(*[c[3] for c in cols])
        rc = self._libh.psvd_pstream_incorporate(self._h, A_ptrs, lds, int(N), cols[0][4])
        _lib.check(rc, self._h, "pstream_incorporate")
        return self

    initialize = incorporate_data

    @property
    def rank(self):
        r = ctypes.c_int32()
        _lib.check(self._libh.psvd_rank(self._h, ctypes.byref(r)), self._h)
        return int(r.value)

    @property
    def singular_values(self):
        r = self.rank
        out = np.zeros(max(r, 1), dtype=np.float64)
        rr = ctypes.c_int32()
        rc = self._libh.psvd_singular_values(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             out.size, ctypes.byref(rr))
        _lib.check(rc, self._h, "singular_values")
        return out[:rr.value].copy()

    def modes_part(self, i):
        """M_i x r modes of partition i (a copy, column-major CUDA tensor)."""
        r = self.rank
        dt = torch.float64 if self.precision == "fp64" else torch.float32
        m = self.M_parts[i]
        out = torch.empty((r, m), dtype=dt, device="cuda")
        if r:
            rc = self._libh.psvd_pstream_modes(self._h, int(i), ctypes.c_void_p(out.data_ptr()), m)
            _lib.check(rc, self._h, "pstream_modes")
        return out.t()

    @property
    def modes(self):
        """Stacked modes (sum M_i x r)."""
        return torch.cat([self.modes_part(i) for i in range(len(self.M_parts))], dim=0)

    def stats(self):
        return StreamingSVD.stats(self)

    def reset_stats(self):
        _lib.check(self._libh.psvd_reset_stats(self._h), self._h)


def rsvd(A, K, oversampling=10, power_iters=2, seed=0, precision="fp32", out_dtype=None, stream=None):
    """One-shot randomized SVD of an M x N CUDA matrix (Eqs. (7)-(11)) -> (U (M x r), s (r,), V (N x r))."""
    lib = _lib.load()
    ptr, M, N, lda, code, keep = _as_colmajor(A)
    dt = out_dtype or (torch.float64 if precision == "fp64" else torch.float32)
    ocode = _lib.PSVD_F64 if dt == torch.float64 else _lib.PSVD_F32
    r = min(int(K), N)
    U = torch.empty((r, M), dtype=dt, device=A.device)
    V = torch.empty((r, N), dtype=dt, device=A.device)
    s = np.zeros(max(int(K), 1), dtype=np.float64)
    rank = ctypes.c_int32()
    rc = lib.psvd_rsvd(ptr, M, N, lda, code, int(K), int(oversampling), int(power_iters), ctypes.c_uint64(int(seed)),
                       _PREC[precision], ctypes.c_void_p(U.data_ptr()), M, ctypes.c_void_p(V.data_ptr()), N, ocode,
                       s.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(rank), _stream_ptr(stream))
    if rc != _lib.PSVD_OK:
        raise PsvdError(rc, "rsvd " + lib.psvd_last_error(None).decode())
    r = int(rank.value)
    return U[:r].t(), s[:r].copy(), V[:r].t()


def rsvd_noalloc(A, K, oversampling=10, power_iters=2, seed=0, precision="fp32", stream=None):
    """psvd_rsvd_noalloc: the one-shot randomized SVD with all device workspace taken
    from the library's fixed scratch array (no allocation inside the call).  The
    outputs U (M x r), V (N x r) are allocated here, by the caller side, in the
    precision's element type."""
    lib = _lib.load()
    ptr, M, N, lda, code, keep = _as_colmajor(A)
    dt = torch.float64 if precision == "fp64" else torch.float32
    ocode = _lib.PSVD_F64 if dt == torch.float64 else _lib.PSVD_F32
    r = min(int(K), N)
    U = torch.empty((r, M), dtype=dt, device=A.device)
    V = torch.empty((r, N), dtype=dt, device=A.device)
    s = np.zeros(max(int(K), 1), dtype=np.float64)
    rank = ctypes.c_int32()
    rc = lib.psvd_rsvd_noalloc(ptr, M, N, lda, code, int(K), int(oversampling), int(power_iters),
                               ctypes.c_uint64(int(seed)), _PREC[precision], ctypes.c_void_p(U.data_ptr()), M,
                               ctypes.c_void_p(V.data_ptr()), N, ocode,
                               s.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(rank),
                               _stream_ptr(stream))
    if rc != _lib.PSVD_OK:
        raise PsvdError(rc, "rsvd_noalloc " + lib.psvd_last_error(None).decode())
    r = int(rank.value)
    return U[:r].t(), s[:r].copy(), V[:r].t()


def apmos_batched(parts, r=50, K=5, stream=None, low_rank_ell=0, seed=0):
    """Algorithm 2 over row partitions (list of M_i x N CUDA tensors, same dtype).

    r, K: the local and global truncations (the paper's defaults r1 = 50 and
    r2 = 5; r is clamped to N).  low_rank_ell > 0: the SVD of W is the paper's
    low-rank SVD with an ell-column test matrix keyed by `seed`
    (psvd_apmos_low_rank).  Returns (U_parts, Lambda, X): U_parts[i] is M_i x K
    (column-major), Lambda the K global singular values, X the N x K right factor.
    """
    lib = _lib.load()
    P = len(parts)
    if P == 0:
        raise ValueError("no partitions")
    cols = [_as_colmajor(p) for p in parts]
    N = cols[0][2]
    code = cols[0][4]
    dt = parts[0].dtype
    outs = [torch.empty((K, c[1]), dtype=dt, device="cuda") for c in cols]
    A_ptrs = (ctypes.c_void_p * P)(*[c[0].value for c in cols])
    Ms = (ctypes.c_int64 * P)(*[c[1] for c in cols])
    lds = (ctypes.c_int64 * P)(*[c[3] for c in cols])
    U_ptrs = (ctypes.c_void_p * P)(*[o.data_ptr() for o in outs])
    ldus = (ctypes.c_int64 * P)(*[c[1] for c in cols])
    Lam = np.zeros(K)
    X = np.zeros((K, N))
    r = min(int(r), N)
    if low_rank_ell:
        rc = lib.psvd_apmos_low_rank(P, A_ptrs, Ms, lds, N, code, r, int(K), int(low_rank_ell),
                                     ctypes.c_uint64(int(seed)), U_ptrs, ldus,
                                     Lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream_ptr(stream))
    else:
        rc = lib.psvd_apmos_batched(P, A_ptrs, Ms, lds, N, code, r, int(K), U_ptrs, ldus,
                                    Lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream_ptr(stream))
    _lib.check(rc, None, "apmos_batched")
    return [o.t() for o in outs], Lam, np.ascontiguousarray(X.T)


def stream_backward(A, batches, K, ff, U_bar, s_bar, stream=None):
    """dL/dA of the deterministic stream given cotangents of its final (U, s) (see psvd.h)."""
    lib = _lib.load()
    ptr, M, Nt, lda, code, keep = _as_colmajor(A)
    dt = A.dtype
    Ub = U_bar.to(dtype=dt).t().contiguous()            # (r, M) -> column-major M x r
    sb = np.ascontiguousarray(np.asarray(s_bar, dtype=np.float64))
    out = torch.empty((Nt, M), dtype=dt, device="cuda")
    rc = lib.psvd_stream_backward(ptr, M, lda, code, int(batches), Nt // int(batches), int(K), float(ff),
                                  ctypes.c_void_p(Ub.data_ptr()), sb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream))
    _lib.check(rc, None, "stream_backward")
    return out.t()


def loss_and_grad(A, batches, K, ff, w, want_grad=True, stream=None):
    """L = ||A - U U^T A||^2 + sum w_j s_j of the deterministic stream, and dL/dA, on the device."""
    lib = _lib.load()
    ptr, M, Nt, lda, code, keep = _as_colmajor(A)
    wv = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    L = ctypes.c_double(0.0)
    out = torch.empty((Nt, M), dtype=A.dtype, device="cuda") if want_grad else None
    rc = lib.psvd_loss_grad(ptr, M, lda, code, int(batches), Nt // int(batches), int(K), float(ff),
                            wv.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(L),
                            ctypes.c_void_p(out.data_ptr()) if want_grad else None, _stream_ptr(stream))
    _lib.check(rc, None, "loss_grad")
    return L.value, (out.t() if want_grad else None)


class StreamingSVDFunction(torch.autograd.Function):
    """(U, s) = deterministic stream of A over `batches` equal batches; backward by the library's adjoint."""

    @staticmethod
    def forward(ctx, A, batches, K, ff):
        M, Nt = A.shape
        svd = StreamingSVD(M, K, ff=ff, precision="fp64" if A.dtype == torch.float64 else "fp32")
        nb = Nt // batches
        for b in range(batches):
            svd.incorporate_data(A[:, b * nb:(b + 1) * nb])
        U = svd.modes.clone()
        s = torch.from_numpy(svd.singular_values).to(A.device)
        svd.close()
        ctx.save_for_backward(A)
        ctx.batches, ctx.K, ctx.ff, ctx.r = batches, K, ff, U.shape[1]
        return U, s

    @staticmethod
    def backward(ctx, U_bar, s_bar):
        (A,) = ctx.saved_tensors
        r = ctx.r   # rank of the forward result (either cotangent may be absent)
        if s_bar is None:
            s_bar = torch.zeros(r, dtype=torch.float64)
        if U_bar is None:
            U_bar = torch.zeros((A.shape[0], r), dtype=A.dtype, device=A.device)
        g = stream_backward(A, ctx.batches, ctx.K, ctx.ff, U_bar, s_bar.detach().double().cpu().numpy())
        return g, None, None, None
