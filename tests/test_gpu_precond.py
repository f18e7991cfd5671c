"""The block-Jacobi factor kept across calls (fpcg_detect_pc): the factor a
launch stores against the oracle's factorisation of the same Gram (eq.
pre_BJ), a store-then-load round trip bitwise equal to a plain launch in every
launch form and block form, and a factor of an earlier channel realisation
(Gauss-Markov step, Sec. V) used on the next one, against the oracle given
the same factor."""
import numpy as np
import pytest

import workload as W
from oracle import detect as D
from tests.gpu_common import col_rel, labels_consistent, oracle_detect, oracle_spread, quantiles

pytestmark = pytest.mark.gpu

U32 = 2.0**-24


def _dev(H, Y, s2, io):
    import torch

    dev = torch.device("cuda:0")
    return (torch.from_numpy(np.ascontiguousarray(H.astype(io))).to(dev),
            torch.from_numpy(np.ascontiguousarray(Y.astype(io))).to(dev),
            torch.from_numpy(np.ascontiguousarray(s2)).to(dev))


def _full_T(Tb, L):
    """(B, K, L) rows of each block's factor -> block-diagonal (B, K, K)."""
    B, K, _ = Tb.shape
    T = np.zeros((B, K, K), dtype=np.complex128)
    for b0 in range(0, K, L):
        T[:, b0:b0 + L, b0:b0 + L] = Tb[:, b0:b0 + L, :]
    return T


def _np(t):
    return t.cpu().numpy()


# (form, schedule, K, Nbs, R, L, variant, io)
ROUND_TRIP = [
    ("fused", "fp64", 32, 128, 14, 4, 2, np.complex128),
    ("fused", "fp64", 16, 64, 5, 8, 1, np.complex128),
    ("fused", "fp16", 32, 128, 14, 8, 0, np.complex64),
    ("fused", "fp16", 32, 100, 17, 4, 2, np.complex64),
    ("fused", "bf16", 64, 256, 14, 8, 2, np.complex64),
    ("fused", "fp8", 128, 512, 14, 16, 0, np.complex64),
    ("fused", "fp16", 128, 300, 9, 16, 1, np.complex64),
    ("slab", "fp16", 64, 256, 14, 4, 2, np.complex64),
    ("slab", "fp32", 60, 200, 14, 4, 2, np.complex64),
    ("slab", "fp64", 64, 256, 14, 4, 2, np.complex128),
    ("slab", "bf16", 64, 256, 20, 4, 1, np.complex64),
    ("slab", "fp32", 64, 256, 14, 16, 2, np.complex64),
    ("slab", "fp16", 64, 256, 14, 8, 2, np.complex64),
    ("slab", "fp16", 128, 512, 14, 16, 2, np.complex64),
    ("slab", "fp32", 56, 200, 20, 8, 2, np.complex128),
    ("slab", "fp32", 128, 512, 14, 16, 2, np.complex128),
]


@pytest.mark.parametrize("case", ROUND_TRIP, ids=[f"{c[0]}-{c[1]}-K{c[2]}-L{c[5]}-v{c[6]}" for c in ROUND_TRIP])
def test_store_then_load_is_bitwise_the_plain_launch(case):
    import torch

    import paper_2504_09820_amd as fp

    form, sched, K, Nbs, R, L, v, io = case
    print(f"case precond round trip {case}", flush=True)
    wl = W.draw(21, Nbs, K, R, 16, 18.0, 0.6, 0.6, seed=K + L + v)
    H, Y, s2 = _dev(wl.H, wl.Y, wl.sigma2, io)
    ctx = fp.Context(0)
    ctx.set_launch_form(form)
    it = 7
    ref = fp.detect(H, Y, s2, 16, it, L, sched, variant=v, ctx=ctx)
    tdt = torch.complex128 if sched == "fp64" else torch.complex64
    T = torch.zeros((21, K, L), dtype=tdt, device=H.device)
    a = fp.detect(H, Y, s2, 16, it, L, sched, variant=v, ctx=ctx, precond=T, precond_mode="store")
    b = fp.detect(H, Y, s2, 16, it, L, sched, variant=v, ctx=ctx, precond=T, precond_mode="load")
    torch.cuda.synchronize()
    for out in (a, b):
        assert np.array_equal(_np(out[0]).view(np.uint8), _np(ref[0]).view(np.uint8))
        assert np.array_equal(_np(out[1]), _np(ref[1]))
    assert np.array_equal(_np(a[2]), _np(ref[2]))
    assert np.all(np.isfinite(_np(T)))
    ctx.close()


@pytest.mark.parametrize("sched,K,Nbs,L,io", [("fp64", 32, 128, 4, np.complex128), ("fp64", 64, 256, 8, np.complex128),
                                              ("fp16", 64, 256, 4, np.complex64), ("fp32", 32, 100, 8, np.complex64),
                                              ("fp32", 64, 256, 16, np.complex64),
                                              ("fp16", 64, 256, 8, np.complex64),
                                              ("fp32", 128, 512, 16, np.complex64)])
def test_stored_factor_matches_the_oracles(sched, K, Nbs, L, io):
    """T = C^{-1} of each diagonal block of the u_W Gram (eq. pre_BJ).  FP64:
    within 1e-12 of the oracle's factor of its Gram; FP32 work: the Gram
    differs from the oracle's by FP32 accumulation order (Thm 1, u = 2^-24),
    which a block of condition number kappa_b moves by about kappa_b times as
    much."""
    import torch

    import paper_2504_09820_amd as fp

    print(f"case stored factor {sched} K={K} L={L}", flush=True)
    wl = W.draw(9, Nbs, K, 3, 16, 15.0, 0.7, 0.7, seed=3 + K + L)
    H, Y, s2 = _dev(wl.H, wl.Y, wl.sigma2, io)
    tdt = torch.complex128 if sched == "fp64" else torch.complex64
    T = torch.zeros((9, K, L), dtype=tdt, device=H.device)
    for form in ("fused", "slab"):
        if form == "slab" and not ((K == 64 and L in (4, 8)) or L == 16):
            continue
        if form == "fused" and L == 16:               # L = 16 in fp32 is built as the slab form only
            continue
        ctx = fp.Context(0)
        ctx.set_launch_form(form)
        fp.detect(H, Y, s2, 16, 2, L, sched, variant=2, ctx=ctx, precond=T, precond_mode="store")
        torch.cuda.synchronize()
        Tg = _full_T(_np(T).astype(np.complex128), L)
        name = {"fp8": "e4m3"}.get(sched, sched)
        A, _ = D.gram(wl.H.astype(io).astype(np.complex128), wl.Y.astype(io).astype(np.complex128), wl.sigma2,
                      D.schedule(name))
        To, bad = D.bj_factor(A, L, "fp64")
        assert not bad.any()
        rel = np.linalg.norm(Tg - To, axis=(-2, -1)) / np.linalg.norm(To, axis=(-2, -1))
        kb = max(np.linalg.cond(A[c, b0:b0 + L, b0:b0 + L]) for c in range(9) for b0 in range(0, K, L))
        tol = 1e-12 if sched == "fp64" else 8 * kb * Nbs**0.5 * U32
        print(f"  {form}: max rel {rel.max():.2e} (tol {tol:.2e}, block kappa {kb:.1f})", flush=True)
        assert rel.max() <= tol
        ctx.close()


@pytest.mark.parametrize("sched,K,Nbs,L,v,iters,io,form", [
    ("fp64", 32, 128, 4, 2, 96, np.complex128, "fused"),
    ("fp64", 32, 128, 8, 1, 96, np.complex128, "fused"),
    ("fp16", 32, 128, 4, 2, 11, np.complex64, "fused"),
    ("fp16", 64, 256, 4, 2, 16, np.complex64, "slab"),
    ("fp16", 32, 128, 8, 0, 11, np.complex64, "fused"),
    ("fp32", 128, 512, 16, 2, 24, np.complex64, "slab"),
    ("fp16", 64, 256, 8, 2, 16, np.complex64, "slab"),
])
def test_factor_of_the_previous_interval_on_the_next(sched, K, Nbs, L, v, iters, io, form):
    """Gauss-Markov step (rho = J0(2 pi 1 kHz / 14 kHz)): the factor stored for
    step 0 drives the solve of step 1.  The oracle, given the same factor,
    is the reference: FP64 at I = 3K within 1e-12 (and, any HPD
    preconditioner leaving the solution unchanged, within 1e-10 of step 1's
    LMMSE solution); fp16 at the timed I within four times the oracle's own
    rounding-order spread."""
    import torch

    import paper_2504_09820_amd as fp

    print(f"case stale factor {sched} K={K} L={L} v{v} I={iters} {form}", flush=True)
    steps = W.gauss_markov(24, Nbs, K, 14, 64, 20.0, 0.5, 0.5, steps=2, fd_hz=1000.0, seed=40 + K + L)
    ctx = fp.Context(0)
    ctx.set_launch_form(form)
    tdt = torch.complex128 if sched == "fp64" else torch.complex64
    H0, Y0, s0 = _dev(steps[0].H, steps[0].Y, steps[0].sigma2, io)
    T = torch.zeros((24, K, L), dtype=tdt, device=H0.device)
    fp.detect(H0, Y0, s0, 64, 2, L, sched, variant=v, ctx=ctx, precond=T, precond_mode="store")
    H1, Y1, s1 = _dev(steps[1].H, steps[1].Y, steps[1].sigma2, io)
    x, lab, fl = fp.detect(H1, Y1, s1, 64, iters, L, sched, variant=v, ctx=ctx, precond=T, precond_mode="load")
    torch.cuda.synchronize()
    x = _np(x).astype(np.complex128)
    Tg = _full_T(_np(T).astype(np.complex128), L)
    wl1 = steps[1]
    if sched == "fp64":
        ref = oracle_detect(wl1, 64, iters, L, "fp64", io, variant=v, T_given=Tg)
        assert np.max(col_rel(x, ref.xhat)) < 1e-12
        A1, b1 = D.gram(wl1.H, wl1.Y, wl1.sigma2)
        assert np.max(col_rel(x, D.lmmse(A1, b1))) < 1e-10
    else:
        spread, ref = oracle_spread(wl1, 64, iters, L, sched, io, variant=v, T_given=Tg)
        nrm = np.linalg.norm(ref.xhat, axis=-2)
        qg = quantiles(np.linalg.norm(x - ref.xhat, axis=-2) / nrm)
        qs = quantiles(spread / nrm)
        print(f"  gpu-oracle {qg}  oracle spread {qs}", flush=True)
        assert np.all(qg <= 4.0 * qs + 18 * U32)
        ok, _, _ = labels_consistent(_np(lab), ref.labels, x, ref.xhat, 64, x_alt=ref.x_alt)
        assert ok
    assert np.array_equal(_np(fl), ref.flags.astype(np.int32))
    ctx.close()


def test_precond_arguments_rejected():
    import torch

    import paper_2504_09820_amd as fp

    wl = W.draw(4, 64, 16, 2, 16, 15.0, 0.5, 0.5, seed=1)
    H, Y, s2 = _dev(wl.H, wl.Y, wl.sigma2, np.complex64)
    T = torch.zeros((4, 16, 4), dtype=torch.complex64, device=H.device)
    with pytest.raises(ValueError):
        fp.detect(H, Y, s2, 16, 4, 0, "fp16", precond=T, precond_mode="store")       # L = 0
    with pytest.raises(ValueError):
        fp.detect(H, Y, s2, 16, 4, 4, "fp16", precond=T, precond_mode="keep")
    with pytest.raises(TypeError):
        fp.detect(H, Y, s2, 16, 4, 4, "fp16", variant=2, precond=T.to(torch.complex128), precond_mode="store")
    with pytest.raises(ValueError):
        fp.detect(H, Y, s2, 16, 4, 4, "fp16", variant=2, precond=T[:, :, :2].contiguous(), precond_mode="store")
