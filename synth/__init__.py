"""Seeded synthetic snapshot matrices with planted spectra.

This module only manufactures inputs: it holds none of the streaming /
randomized / partitioned SVD arithmetic.  Both the GPU library's tests and
benchmark and the FP64 oracle consume what it produces.

Recipe (one torch.Generator per workload, draws in this order):
  1. Phi  = orthonormal columns of a (M_total x R) standard normal matrix,
  2. Cfac = orthonormal columns of a (N_total x R) standard normal matrix,
  3. batch b = Phi diag(sigma) Cfac[b-th block of rows]^T
              + eta * standard normal (M x N_b), drawn batch by batch,
  4. cast to the storage dtype (round to nearest even).
Orthonormalisation is Cholesky-QR applied twice with the small Cholesky on
the host in float64 (positive-diagonal triangular factor), which is exact to
rounding for Gaussian matrices (condition number close to 1).

Layout: every batch is returned as a torch tensor of shape (N_b, M),
contiguous, i.e. the M x N_b matrix in column-major order with each
snapshot contiguous.  `numpy_cm(t)` gives the (M, N_b) Fortran-ordered
float64 view used by the oracle.

The workloads below mirror the five configurations the library is measured
and checked on (sizes, spectra, noise levels, seeds).
"""
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np
import torch


@dataclass
class Workload:
    name: str
    M: int                      # rows (grid points) per batch / total rows for APMOS
    N: int                      # snapshots per batch (columns per partition for APMOS)
    batches: int
    K: int
    oversampling: int = 0
    power_iters: int = 0
    ff: float = 1.0
    sigma: Optional[np.ndarray] = None   # planted spectrum (length R)
    noise: float = 0.0                   # standard deviation of i.i.d. Gaussian noise
    seed: int = 0
    dtype: torch.dtype = torch.float32
    randomized: bool = False
    precision: str = "fp32"              # fp64 | fp32 | mixed
    partitions: int = 0                  # APMOS only
    part_min: int = 0
    part_max: int = 0
    local_rank: int = 0                  # APMOS r
    extra: dict = field(default_factory=dict)


def c1_plain_fp64() -> Workload:
    j = np.arange(20, dtype=np.float64)
    return Workload("streaming_fp64_M4096_N64x4_K10", M=4096, N=64, batches=4, K=10, ff=1.0,
                    sigma=2.0 ** (-j / 2.0), noise=1e-6, seed=0, dtype=torch.float64,
                    randomized=False, precision="fp64")


def c2_randomized_fp32() -> Workload:
    j = np.arange(1, 201, dtype=np.float64)
    return Workload("randomized_streaming_M1048576_N256x16_K50_p10_q2", M=1 << 20, N=256, batches=16,
                    K=50, oversampling=10, power_iters=2, ff=0.95, sigma=j ** -1.5, noise=1e-5, seed=1,
                    dtype=torch.float32, randomized=True, precision="fp32")


def c3_mixed() -> Workload:
    j = np.arange(400, dtype=np.float64)
    return Workload("mixed_streaming_M4194304_N512x8_K100_p20_q1", M=1 << 22, N=512, batches=8, K=100,
                    oversampling=20, power_iters=1, ff=0.95, sigma=np.exp(-j / 30.0), noise=0.0, seed=2,
                    dtype=torch.float32, randomized=True, precision="mixed")


def c4_apmos() -> Workload:
    j = np.arange(40, dtype=np.float64)
    return Workload("apmos_P64_N128_r20_K20", M=0, N=128, batches=1, K=20, sigma=2.0 ** (-j / 3.0), noise=0.0,
                    seed=3, dtype=torch.float32, partitions=64, part_min=16384, part_max=262144, local_rank=20)


def c5_gradient() -> Workload:
    j = np.arange(1, 257, dtype=np.float64)
    s20 = 2.0 ** (-(20 - 1) / 4.0)
    sig = np.where(j <= 20, 2.0 ** (-(j - 1) / 4.0), (s20 / 4.0) * 2.0 ** (-(j - 21) / 8.0))
    return Workload("gradient_M262144_N64x4_K20", M=1 << 18, N=64, batches=4, K=20, ff=1.0, sigma=sig,
                    noise=0.0, seed=4, dtype=torch.float32, randomized=False, precision="fp32")


ALL = {"c1": c1_plain_fp64, "c2": c2_randomized_fp32, "c3": c3_mixed, "c4": c4_apmos, "c5": c5_gradient}


def scaled(w: Workload, **kw) -> Workload:
    """Copy of a workload with some fields replaced (e.g. a smaller M for the oracle)."""
    return replace(w, **kw)


def _orthonormal(rows: int, cols: int, gen: torch.Generator, device) -> torch.Tensor:
    """Orthonormal columns spanning a standard normal rows x cols draw (float64)."""
    X = torch.randn((rows, cols), generator=gen, dtype=torch.float64, device=device)
    for _ in range(2):
        G = (X.T @ X).cpu()
        L = torch.linalg.cholesky(G)                   # G = L L^T, L_jj > 0
        Linv_T = torch.linalg.inv(L).T.contiguous()    # X L^-T has orthonormal columns
        X = X @ Linv_T.to(device)
    return X


def planted_stream(w: Workload, device="cpu", batches: Optional[int] = None) -> List[torch.Tensor]:
    """Batches of the planted-spectrum stream: list of (N, M) tensors (column-major M x N)."""
    nb = w.batches if batches is None else batches
    gen = torch.Generator(device=device)
    gen.manual_seed(int(w.seed))
    # A planted spectrum longer than the matrix allows is cut to min(M, N_total) modes.
    R = min(len(w.sigma), w.M, w.N * w.batches)
    sig = torch.as_tensor(np.asarray(w.sigma[:R], dtype=np.float64), device=device)
    Phi = _orthonormal(w.M, R, gen, device)
    Cf = _orthonormal(w.N * w.batches, R, gen, device)
    PhiS_T = (Phi * sig).T.contiguous()                # R x M
    del Phi
    out = []
    for b in range(nb):
        At = Cf[b * w.N:(b + 1) * w.N] @ PhiS_T        # (N, M) float64
        if w.noise > 0:
            At += w.noise * torch.randn((w.N, w.M), generator=gen, dtype=torch.float64, device=device)
        out.append(At.to(w.dtype).contiguous())
        del At
    return out


def partition_sizes(w: Workload) -> List[int]:
    """Row counts of the APMOS partitions, uniform integers in [part_min, part_max] (drawn first)."""
    rng = np.random.default_rng(w.seed)
    return [int(x) for x in rng.integers(w.part_min, w.part_max + 1, size=w.partitions)]


def apmos_partitions(w: Workload, device="cpu", sizes: Optional[List[int]] = None) -> List[torch.Tensor]:
    """Row partitions of one planted matrix A = Phi diag(sigma) C^T (sum M_i x N); list of (N, M_i) tensors."""
    if sizes is None:
        sizes = partition_sizes(w)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(w.seed) + 1000)
    Mt = int(sum(sizes))
    R = min(len(w.sigma), Mt, w.N)
    sig = torch.as_tensor(np.asarray(w.sigma[:R], dtype=np.float64), device=device)
    Phi = _orthonormal(Mt, R, gen, device)
    Cf = _orthonormal(w.N, R, gen, device)
    CS = (Cf * sig)                                    # N x R
    out, off = [], 0
    for m in sizes:
        At = CS @ Phi[off:off + m].T                   # (N, m)
        if w.noise > 0:
            At += w.noise * torch.randn((w.N, m), generator=gen, dtype=torch.float64, device=device)
        out.append(At.to(w.dtype).contiguous())
        off += m
    return out


def loss_weights(w: Workload) -> np.ndarray:
    """Weights w_j ~ U(0, 1) of the differentiable loss (drawn after the data)."""
    rng = np.random.default_rng(w.seed + 7)
    return rng.uniform(0.0, 1.0, size=w.K)


def numpy_cm(t: torch.Tensor) -> np.ndarray:
    """(N, M) contiguous tensor -> (M, N) float64 Fortran-ordered numpy array (same column-major matrix)."""
    return np.asfortranarray(t.detach().to("cpu", torch.float64).numpy().T)


def burgers_snapshots(nx: int = 16384, nt: int = 800, Re: float = 1000.0, L: float = 1.0, tf: float = 2.0,
                      dtype=torch.float64, device="cpu") -> torch.Tensor:
    """Snapshots of the viscous Burgers equation from its closed-form solution
    (the paper's first experiment, Eq. (13)): u(x, t) = (x / (t + 1)) /
    (1 + sqrt((t + 1) / t0) exp(Re x^2 / (4 t + 4))), t0 = exp(Re / 8), on nx
    equispaced points of [0, L] and nt equispaced times of [0, tf].

    Evaluated in float64 with the square root folded into the exponent
    (exp(Re x^2 / (4t + 4) + ln(t + 1) / 2 - Re / 16)), whose largest
    argument (x = L, t = 0) is Re / 4 - Re / 16, finite in float64; then cast
    to `dtype`.  Returns an (nt, nx) tensor: the nx x nt snapshot matrix in
    column-major order (one snapshot per column)."""
    x = torch.linspace(0.0, L, nx, dtype=torch.float64, device=device)
    t = torch.linspace(0.0, tf, nt, dtype=torch.float64, device=device)[:, None]
    e = Re * x[None, :] ** 2 / (4.0 * t + 4.0) + 0.5 * torch.log(t + 1.0) - Re / 16.0
    u = (x[None, :] / (t + 1.0)) / (1.0 + torch.exp(e))
    return u.to(dtype).contiguous()
