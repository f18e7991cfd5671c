"""Host-side precision selection (eq. heuristic and eq. heuristic_bj).

The heuristic asks for u_MV < 1 / (N^1.5 sqrt(kappa)) with kappa the expected
condition number of the system the iteration runs on: A for FP-CG, the
block-Jacobi preconditioned matrix for FP-BJ-CG (whose spectrum is that of
T A T^H with T = blockdiag(C_i^{-1}), A_i = C_i C_i^H).  kappa is estimated
once per workload class from a sample of its channels (the expectation that
the heuristic's footnote allows), then the library's fpcg_select_precision
picks the cheapest format below the bound.  This is calibration done on the
host before any detection; nothing here runs per channel on the hot path.
"""
from __future__ import annotations

import numpy as np


def expected_kappa(H, sigma2, L: int = 0, sample: int = 64, seed: int = 0) -> float:
    """Mean 2-norm condition number over up to `sample` channels of A = H^H H +
    sigma^2 I (L = 0) or of T A T^H with L x L Jacobi blocks (L > 0).
    H is (B, Nbs, K) complex (numpy or a CPU-copyable tensor), sigma2 (B,)."""
    H = np.asarray(H.cpu() if hasattr(H, "cpu") else H)
    s2 = np.asarray(sigma2.cpu() if hasattr(sigma2, "cpu") else sigma2, dtype=np.float64)
    B, _, K = H.shape
    idx = np.random.default_rng(seed).choice(B, size=min(sample, B), replace=False)
    kap = []
    for c in idx:
        h = H[c].astype(np.complex128)
        a = h.conj().T @ h + s2[c] * np.eye(K)
        if L > 0:
            t = np.zeros_like(a)
            for b in range(0, K, L):
                ch = np.linalg.cholesky(a[b:b + L, b:b + L])
                t[b:b + L, b:b + L] = np.linalg.solve(ch, np.eye(L))
            a = t @ a @ t.conj().T
        ev = np.linalg.eigvalsh(a)
        kap.append(ev[-1] / ev[0])
    return float(np.mean(kap))


def choose_format(K: int, kappa: float, allow_fp8: bool = False) -> tuple[str, float]:
    """(format name, u bound) the heuristic selects for a K-dimensional system."""
    from . import select_precision

    return select_precision(K, kappa, allow_fp8)
