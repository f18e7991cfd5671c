"""Analysis results of the paper used as test pins and for precision selection.

TEST INFRASTRUCTURE ONLY (see the package docstring).

  gamma(n, u)             eq. gamma: gamma_n = n u / (1 - n u)
  attainable_bound(...)   Thm 2 (eq. mp) / Thm 4 (eq. bj_mp): bound on
                          ||b - A x_i - r_i|| / (||A|| ||x||)
  heuristic_bound(N, k)   eq. heuristic / eq. heuristic_bj: u_MV < 1/(N^1.5 sqrt(kappa))
  select_format(N, k)     pick the cheapest format of Table I (plus fp8) below it
  gram_entry_variance     App. B, eq. var: variance of an off-diagonal Gram entry
  cost model              Sec. V-A: real multiplications weighted fp16:fp32:fp64 =
                          1:2:4, counting A p, M_d r, the BJ setup and the direct
                          inverse (the model that reproduces the paper's
                          percentages in Sec. V-C and App. E)
"""
from __future__ import annotations

import math

import numpy as np

from .rounding import UNIT_ROUNDOFF


def gamma(n: int, u: float) -> float:
    """eq. gamma."""
    nu = n * u
    if nu >= 1:
        return math.inf
    return nu / (1.0 - nu)


def upsilon(i: int, N: int, u_w: float, u_mv: float) -> float:
    """Upsilon_i of Thm 2: ((8 sqrt2 + 6) i + 1) u_W + (2 i + 1) 2 sqrt2 N^1.5 u_MV."""
    return ((8.0 * math.sqrt(2.0) + 6.0) * i + 1.0) * u_w + (2.0 * i + 1.0) * 2.0 * math.sqrt(2.0) * N ** 1.5 * u_mv


def attainable_bound(i: int, N: int, u_w: float, u_mv: float, theta: float) -> float:
    """eq. mp / eq. bj_mp: (1 + i) u_W + Upsilon_i Theta_i."""
    return (1.0 + i) * u_w + upsilon(i, N, u_w, u_mv) * theta


def residual_gap(A, b, x_i, r_i, x_true):
    """Left-hand side of eq. mp for every column: ||b - A x_i - r_i|| / (||A||_2 ||x||)."""
    num = np.linalg.norm(b - A @ x_i - r_i, axis=-2)
    an = np.linalg.norm(A, ord=2, axis=(-2, -1))[..., None]
    return num / (an * np.linalg.norm(x_true, axis=-2))


def heuristic_bound(N: int, kappa: float) -> float:
    """eq. heuristic (kappa of A) / eq. heuristic_bj (kappa of the preconditioned A)."""
    return 1.0 / (N ** 1.5 * math.sqrt(kappa))


# candidate operand formats in order of increasing cost; equal-cost candidates in
# order of increasing unit roundoff (fp16 before bf16: same matrix-core rate,
# three more significand bits)
_CANDIDATES = [("e4m3", 0.5), ("fp16", 1.0), ("bf16", 1.0), ("fp32", 2.0), ("fp64", 4.0)]


def select_format(N: int, kappa: float, allow_fp8: bool = True) -> str:
    """Cheapest format whose unit roundoff satisfies the heuristic."""
    bound = heuristic_bound(N, kappa)
    for name, _cost in _CANDIDATES:
        if name == "e4m3" and not allow_fp8:
            continue
        if UNIT_ROUNDOFF[name] < bound:
            return name
    return "fp64"


def expected_kappa(H_batch, sigma2, L: int = 0) -> float:
    """Monte-Carlo E{kappa} of A (L = 0) or of the BJ-preconditioned A (L > 0)."""
    H = np.asarray(H_batch)
    K = H.shape[-1]
    s2 = np.asarray(sigma2, dtype=np.float64).reshape(-1, 1, 1)
    A = np.conj(np.swapaxes(H, -1, -2)) @ H + s2 * np.eye(K)
    ks = []
    for a in A:
        if L:
            ch = np.zeros_like(a)
            for j in range(K // L):
                sl = slice(j * L, (j + 1) * L)
                ch[sl, sl] = np.linalg.cholesky(a[sl, sl])
            ci = np.linalg.inv(ch)
            a = ci @ a @ ci.conj().T
        w = np.linalg.eigvalsh(a)
        ks.append(w[-1] / w[0])
    return float(np.mean(ks))


def gram_entry_variance(M: int, zeta: float) -> float:
    """App. B, eq. var: V{h_n^H h_i} = 1/M + (2/M^2) [s (M-1) - s^2 (1 - zeta^(2(M-1)))],
    s = zeta^2 / (1 - zeta^2), for CN(0, 1/M) entries and BS-side correlation zeta."""
    s = zeta * zeta / (1.0 - zeta * zeta)
    return 1.0 / M + 2.0 / M**2 * (s * (M - 1) - s * s * (1.0 - zeta ** (2 * (M - 1))))


# --------------------------------------------------------------------------
# cost model (Sec. V-A ratio 1:2:4; counts real multiplications, 4 per complex one)
# --------------------------------------------------------------------------
COST_WEIGHT = {"fp16": 1.0, "bf16": 1.0, "fp32": 2.0, "fp64": 4.0, "e4m3": 0.5}


def cost_cg(N: int, iters: int, u_mv: str = "fp64") -> float:
    """CG / FP-CG: per iteration the N x N complex product A p at u_MV."""
    return iters * 4.0 * N * N * COST_WEIGHT[u_mv]


def cost_bj_setup(N: int, L: int, u: str = "fp64") -> float:
    """BJ setup: d = N/L inverses of L x L blocks, N L^2 complex multiplications."""
    return 4.0 * N * L * L * COST_WEIGHT[u]


def cost_bj_cg(N: int, L: int, iters: int, u_mv: str = "fp16", u_w: str = "fp64") -> float:
    """FP-BJ-CG: setup + per iteration A p at u_MV and M_d r (N L complex) at u_W."""
    per_it = 4.0 * N * N * COST_WEIGHT[u_mv] + 4.0 * N * L * COST_WEIGHT[u_w]
    return cost_bj_setup(N, L, u_w) + iters * per_it


def cost_lmmse(N: int, u: str = "fp64") -> float:
    """Direct inverse of the N x N Gram: N^3 complex multiplications."""
    return 4.0 * N**3 * COST_WEIGHT[u]


def reduction(cost, reference) -> float:
    """Relative saving 1 - cost / reference, in percent."""
    return 100.0 * (1.0 - cost / reference)
