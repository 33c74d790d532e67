import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests are skipped (not failed) when no GPU is visible, so a plain
    # `pytest` on a CPU-only machine stays green; `-m gpu` on a machine with a GPU runs them.
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


# ----------------------------------------------------------------------------
# Comparison helpers shared by the oracle pins and the GPU parity tests.
# ----------------------------------------------------------------------------

def sigma_rel_err(s_hat, s_ref, n=None, u=2.0 ** -53):
    """max_j |s_hat_j - s_ref_j| / s_ref_j over modes above the numerical-rank floor n*u*s_1."""
    s_hat = np.asarray(s_hat, dtype=np.float64)
    s_ref = np.asarray(s_ref, dtype=np.float64)
    k = min(len(s_hat), len(s_ref))
    s_hat, s_ref = s_hat[:k], s_ref[:k]
    if k == 0:
        return 0.0
    floor = (n if n is not None else k) * u * s_ref[0]
    m = s_ref > floor
    if not np.any(m):
        return 0.0
    return float(np.max(np.abs(s_hat[m] - s_ref[m]) / s_ref[m]))


def max_principal_angle(U1, U2):
    """Largest principal angle (radians) between span(U1) and span(U2) (orthonormal columns)."""
    U1 = np.asarray(U1, dtype=np.float64)
    U2 = np.asarray(U2, dtype=np.float64)
    if U1.shape[1] == 0:
        return 0.0
    sv = np.linalg.svd(U1.T @ U2, compute_uv=False)
    c = np.clip(sv.min(), -1.0, 1.0)
    # arccos loses accuracy near 1: use the sine from the complement instead.
    P = U2 - U1 @ (U1.T @ U2)
    s = np.linalg.svd(P, compute_uv=False).max() if P.size else 0.0
    return float(min(np.arccos(c), np.arcsin(min(1.0, s))))


def orth_err(U):
    U = np.asarray(U, dtype=np.float64)
    k = U.shape[1]
    return float(np.linalg.norm(U.T @ U - np.eye(k)))


def gap_limited_k(s, tol, kmax):
    """Largest k <= kmax whose relative gap (s_k - s_{k+1}) / s_1 >= 1e3 * tol (leading modes only)."""
    s = np.asarray(s, dtype=np.float64)
    best = 0
    for k in range(1, min(kmax, len(s) - 1) + 1):
        if (s[k - 1] - s[k]) / s[0] >= 1e3 * tol:
            best = k
    return best


def align_signs(U_hat, U_ref):
    """Flip columns of U_hat to best match U_ref (sign ambiguity of singular vectors)."""
    U_hat = np.array(U_hat, dtype=np.float64, copy=True)
    for j in range(min(U_hat.shape[1], U_ref.shape[1])):
        if np.dot(U_hat[:, j], U_ref[:, j]) < 0:
            U_hat[:, j] = -U_hat[:, j]
    return U_hat
