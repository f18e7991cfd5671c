"""Precision selection (eq. heuristic and eq. heuristic_bj).

The heuristic asks for u_MV < 1 / (N^1.5 sqrt(kappa)) with kappa the expected
condition number of the system the iteration runs on: A for FP-CG, the
block-Jacobi preconditioned matrix for FP-BJ-CG.  kappa is estimated once per
workload class on the device from a sample of its channels (the expectation
that the heuristic's footnote allows; fpcg_expected_kappa), then the
library's fpcg_select_precision picks the cheapest format below the bound.
The context keeps the estimate, so a detection with no schedule
(detect(..., schedule_=None)) runs in the heuristic's format.  Nothing here
does the method's arithmetic: the helpers below only marshal the library's
calls and apply the scalar bound.

Per channel (the alternative the footnote also allows): a detection with a
kappa output (fpcg_detect_ex) estimates each channel's kappa from its CG
coefficients; formats_per_channel() applies the same bound to each estimate
and detect_adaptive() runs each group of channels in its format, one
launch per format over that group's channel indices (H and Y stay where
they are).
"""
from __future__ import annotations

import numpy as np


def expected_kappa(H, Y, sigma2, L: int = 0, sample: int = 64, ctx=None) -> float:
    """E{kappa} of the iteration matrix of A = H^H H + sigma^2 I (L = 0) or of
    its block-Jacobi preconditioned form (L > 0), estimated on the device from
    up to `sample` channels spread over the batch (fpcg_expected_kappa) and
    recorded in the context.  H (B, Nbs, K), Y (B, Nbs, R) complex and sigma2
    (B,) float64: CUDA tensors, or numpy arrays copied to the device."""
    import torch

    from . import _ctx_for

    dev = torch.device("cuda", ctx.device) if ctx is not None else torch.device("cuda:0")

    def on_dev(a, dtype=None):
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a))
        return a.to(dev, dtype=dtype) if dtype is not None else a.to(dev)

    H = on_dev(H)
    Y = on_dev(Y, H.dtype)
    s2 = on_dev(sigma2, torch.float64)
    ctx = ctx or _ctx_for(dev.index or 0)
    return ctx.expected_kappa(H, Y, s2, L, sample)


def choose_format(K: int, kappa: float, allow_fp8: bool = False) -> tuple[str, float]:
    """(format name, u bound) the heuristic selects for a K-dimensional system."""
    from . import select_precision

    return select_precision(K, kappa, allow_fp8)


FORMATS = ("fp8", "fp16", "bf16", "fp32", "fp64")


def formats_per_channel(kappa, K: int, allowed=("fp16", "fp32", "fp64"), fallback: str = "fp64") -> np.ndarray:
    """Per channel, the cheapest format in `allowed` whose unit roundoff meets
    u < 1 / (K^1.5 sqrt(kappa)); channels without an estimate (NaN) or with
    none of `allowed` meeting the bound get `fallback`.  Returns an object
    array of format names."""
    u = {"fp8": 2.0 ** -4, "fp16": 2.0 ** -11, "bf16": 2.0 ** -8, "fp32": 2.0 ** -24, "fp64": 2.0 ** -53}
    order = [f for f in FORMATS if f in allowed]
    k = np.asarray(kappa.cpu() if hasattr(kappa, "cpu") else kappa, dtype=np.float64)
    bound = 1.0 / (float(K) ** 1.5 * np.sqrt(np.where(np.isfinite(k) & (k >= 1.0), k, np.nan)))
    out = np.full(k.shape, fallback, dtype=object)
    done = ~np.isfinite(bound)
    for f in order:
        pick = ~done & (u[f] < bound)
        out[pick] = f
        done |= pick
    return out


def detect_adaptive(H, Y, sigma2, qam: int, iters: int, L: int, formats, variant: int = 2, ctx=None, stream=None,
                    out=None):
    """Detect every channel in its own format: one fpcg_detect_ex launch per
    distinct format over that format's channel indices.  `formats` is a
    length-B sequence of format names (formats_per_channel).  Returns
    (xhat, labels, flags, groups) with groups {format: number of channels}."""
    import torch

    from . import detect

    B, _, K = H.shape
    R = Y.shape[2]
    f = np.asarray(formats, dtype=object)
    if f.shape != (B,):
        raise ValueError("one format per channel")
    if out is None:
        out = (torch.empty((B, K, R), dtype=H.dtype, device=H.device),
               torch.empty((B, K, R), dtype=torch.uint8, device=H.device),
               torch.empty((B,), dtype=torch.int32, device=H.device))
    groups = {}
    for name in FORMATS:
        sel = np.nonzero(f == name)[0]
        if sel.size == 0:
            continue
        idx = torch.from_numpy(sel.astype(np.int32)).to(H.device)
        detect(H, Y, sigma2, qam, iters, L, name, variant=variant if L else 0, ctx=ctx, stream=stream, out=out,
               chan_idx=idx)
        groups[name] = int(sel.size)
    return out[0], out[1], out[2], groups


# ---------------------------------------------------------------- block size
def cg_iterations(kappa: float, eps: float = 1e-3) -> int:
    """Steps after which the classical CG error bound 2 ((sqrt(k) - 1) /
    (sqrt(k) + 1))^i (A-norm, relative) drops below eps."""
    if not kappa >= 1.0:
        raise ValueError("kappa must be >= 1")
    if kappa == 1.0:
        return 1
    s = np.sqrt(kappa)
    return int(np.ceil(np.log(2.0 / eps) / np.log((s + 1.0) / (s - 1.0))))


def bj_setup_over_iteration(K: int, L: int) -> float:
    """C_BJ / C^it of Remark 4 with its scalings made exact as in Remark 5:
    N L^2 multiplications for the block inverses against N^2 for the
    iteration's A p (N = K): L^2 / K (K = 32, L = 8 gives 2 iterations)."""
    return (L * L) / K if L else 0.0


def choose_block_size(K: int, kappas: dict | None = None, eps: float = 1e-3, setup_cost=bj_setup_over_iteration,
                      iters: dict | None = None):
    """Block size by the break-even rule of Remark 4: with k(L) the iterations
    needed on the system preconditioned with L x L blocks (L = 0 for none),
    preconditioning with L pays when k(0) - k(L) > C_BJ(L) / C^it.  k(L) is
    either measured (`iters`, {L: k}, e.g. the iteration counts of a
    BER-parity search) or taken from the classical CG bound for the kappa of
    that system (`kappas`, {L: kappa}).  Returns (L, {L: total cost in
    iterations}) with the smallest total (the smaller L on a tie).
    `setup_cost(K, L)` gives C_BJ / C^it; the default is the paper's
    multiplication count, a measured ratio of the device's setup and
    iteration times can be passed instead."""
    if iters is None:
        if kappas is None:
            raise ValueError("pass kappas or iters")
        iters = {L: cg_iterations(k, eps) for L, k in kappas.items()}
    total = {L: setup_cost(K, L) + k for L, k in iters.items()}
    best = min(sorted(total), key=lambda L: total[L])
    return best, total
