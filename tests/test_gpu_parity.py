"""GPU parity of the fused HIP detector against the CPU oracle, through the
C-ABI binding.  Sizes span several 16x16 tiles and ragged tails; the last
tests run the full-size workloads in the benchmark's launch configuration and
compare sampled channels.  The tolerance model is described in gpu_common."""
import sys

import numpy as np
import pytest

import workload as W
from oracle import detect as D
from tests.gpu_common import (boundary_distance, col_rel, gpu_detect, labels_consistent, oracle_detect,
                              oracle_spread, quantiles)

pytestmark = pytest.mark.gpu

U32 = 2.0**-24
# quantile factor of the GPU/oracle distance over the oracle's own order
# sensitivity (the GPU accumulates in a third valid order).  For fp8 operands
# the oracle's second order reproduces the coarser grouped accumulation of
# the fp8 matrix core (each group of 8 products is aligned to its largest
# product and truncated 13 bits below it, measured on the device).
FACTOR = {"fp64": 4.0, "fp32": 4.0, "bf16": 4.0, "fp16": 4.0, "fp8": 4.0}
FLOOR = {"fp64": 1e-13, "fp32": 16 * U32, "bf16": 16 * U32, "fp16": 16 * U32, "fp8": 16 * U32}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _wl(B, Nbs, K, R, q, snr, zeta, seed, norm="paper"):
    return W.draw(B, Nbs, K, R, q, snr, zeta, zeta, seed=seed, normalization=norm)


def _spread_parity(x, ref, spread, sched, tag="", io=np.complex128):
    """x is returned in the I/O element type: compare with the oracle's result
    rounded to that type (complex64 output rounds the FP64 path's x)."""
    ref_x = ref.xhat.astype(io).astype(np.complex128)
    nrm = np.linalg.norm(ref.xhat, axis=-2)
    d = np.linalg.norm(x - ref_x, axis=-2) / nrm
    qg = quantiles(d)
    qs = quantiles(spread / nrm)
    floor = FLOOR[sched] + (2 * U32 if io == np.complex64 else 0.0)
    _say(f"  {tag} gpu-oracle (median, q90, max) {qg}  oracle order spread {qs}")
    assert np.all(qg <= FACTOR[sched] * qs + floor), (qg, qs)


# --------------------------------------------------------------- converged / exact-arithmetic limits
def test_fp64_c1_matches_oracle_to_1e12():
    wl = _wl(37, 64, 8, 1, 16, 10.0, 0.0, 1, "unit")
    _say("case c1 shape, fp64, I=K=8")
    x, lab, fl = gpu_detect(wl, 16, 8, 0, "fp64")
    ref = oracle_detect(wl, 16, 8, 0, "fp64")
    assert np.max(col_rel(x, ref.xhat)) < 1e-12
    assert np.array_equal(lab, ref.labels)
    assert not fl.any()


@pytest.mark.parametrize("K,L,Nbs,variant", [(32, 0, 128, 0), (32, 8, 128, 0), (64, 0, 256, 0), (64, 8, 256, 0),
                                             (20, 4, 50, 0), (32, 8, 128, 2), (64, 8, 256, 2), (20, 4, 50, 2)])
def test_fp64_converged_matches_oracle_to_1e12(K, L, Nbs, variant):
    wl = _wl(6, Nbs, K, 14, 64, 20.0, 0.5, 2)
    iters = 3 * K
    _say(f"case fp64 converged K={K} L={L} variant={variant} I={iters}")
    x, lab, fl = gpu_detect(wl, 64, iters, L, "fp64", variant=variant)
    ref = oracle_detect(wl, 64, iters, L, "fp64", variant=variant)
    assert np.max(col_rel(x, ref.xhat)) < 1e-12
    ok, n, bad = labels_consistent(lab, ref.labels, x, ref.xhat, 64, x_alt=getattr(ref, "x_alt", None))
    assert ok, (n, bad)


@pytest.mark.parametrize("L,variant", [(0, 0), (4, 0), (8, 0), (8, 2)])
def test_fp32_converged_within_1e5_of_lmmse(L, variant):
    wl = _wl(8, 128, 32, 14, 64, 20.0, 0.5, 3)
    _say(f"case fp32 converged L={L} variant={variant}")
    x, lab, fl = gpu_detect(wl, 64, 64, L, "fp32", np.complex64, variant=variant)
    A, b = D.gram(wl.H.astype(np.complex64).astype(np.complex128), wl.Y.astype(np.complex64).astype(np.complex128),
                  wl.sigma2)
    xs = D.lmmse(A, b)
    e = col_rel(x, xs)
    _say(f"  max rel error vs LMMSE {e.max():.2e}")
    assert e.max() < 1e-5
    d = boundary_distance(xs, 64)
    must = d > 1e-3
    assert np.array_equal(lab[must], D.slice_qam(xs, 64)[must])


@pytest.mark.parametrize("sched", ["fp16", "bf16"])
def test_refresh_converges_to_fp32_accuracy(sched):
    wl = _wl(6, 256, 64, 14, 64, 15.0, 0.7, 4)
    _say(f"case {sched} + FP64 refresh converged")
    x, lab, fl = gpu_detect(wl, 64, 64, 8, sched, np.complex64, refresh=4)
    ref = oracle_detect(wl, 64, 64, 8, sched, np.complex64, refresh=4)
    A, b = D.gram(wl.H.astype(np.complex64).astype(np.complex128), wl.Y.astype(np.complex64).astype(np.complex128),
                  wl.sigma2)
    xs = D.lmmse(A, b)
    eg, eo = col_rel(x, xs), col_rel(ref.xhat, xs)
    _say(f"  err vs LMMSE gpu median {np.median(eg):.2e} max {eg.max():.2e}; oracle {np.median(eo):.2e} {eo.max():.2e}")
    assert np.median(eg) <= 2 * np.median(eo) + 1e-6
    assert eg.max() <= 4 * eo.max() + 1e-6


# --------------------------------------------------------------- short horizon: tight
SHORT_MED = {"fp64": 1e-14, "fp32": 2e-6, "bf16": 2e-6, "fp16": 2e-6, "fp8": 5e-5}
SHORT_MAX = {"fp64": 1e-13, "fp32": 1e-5, "bf16": 1e-3, "fp16": 1e-3, "fp8": 1e-2}


@pytest.mark.parametrize("sched", ["fp64", "fp32", "bf16", "fp16", "fp8"])
@pytest.mark.parametrize("L,variant", [(0, 0), (8, 0), (8, 2)])
def test_short_horizon_parity(sched, L, variant):
    io = np.complex128 if sched == "fp64" else np.complex64
    wl = _wl(10, 128, 32, 14, 64, 20.0, 0.5, 5)
    for it in (1, 2):
        x, lab, fl = gpu_detect(wl, 64, it, L, sched, io, variant=variant)
        ref = oracle_detect(wl, 64, it, L, sched, io, variant=variant)
        e = col_rel(x, ref.xhat)
        _say(f"case short {sched} L={L} v{variant} I={it}: median {np.median(e):.2e} max {e.max():.2e}")
        assert np.median(e) <= SHORT_MED[sched] * it and e.max() <= SHORT_MAX[sched] * it


# --------------------------------------------------------------- fixed iteration counts (the configs' shapes)
CASES = [
    # name, B, Nbs, K, R, q, snr, zeta, iters, L, sched, io, refresh, variant
    ("c2-fp64", 8, 128, 32, 14, 64, 20.0, 0.5, 16, 0, "fp64", np.complex128, 0, 0),
    ("c2-fp32", 8, 128, 32, 14, 64, 20.0, 0.5, 16, 0, "fp32", np.complex64, 0, 0),
    ("c2-bf16", 8, 128, 32, 14, 64, 20.0, 0.5, 16, 0, "bf16", np.complex64, 0, 0),
    ("c2-fp16", 8, 128, 32, 14, 64, 20.0, 0.5, 16, 0, "fp16", np.complex64, 0, 0),
    ("c2-fp8", 8, 128, 32, 14, 64, 20.0, 0.5, 16, 0, "fp8", np.complex64, 0, 0),
    ("c2-bf16-c128", 6, 128, 32, 14, 64, 20.0, 0.5, 12, 0, "bf16", np.complex128, 0, 0),
    ("c3-fp64-L8", 5, 256, 64, 14, 64, 15.0, 0.7, 24, 8, "fp64", np.complex128, 0, 0),
    ("c3-fp16-L8-refresh4", 5, 256, 64, 14, 64, 15.0, 0.7, 16, 8, "fp16", np.complex64, 4, 0),
    ("c3-fp16-L4-refresh4", 5, 256, 64, 14, 64, 15.0, 0.7, 16, 4, "fp16", np.complex64, 4, 0),
    ("c3-fp16-L8-textbook", 5, 256, 64, 14, 64, 15.0, 0.7, 16, 8, "fp16", np.complex64, 0, 1),
    ("c3-fp32-L8", 5, 256, 64, 14, 64, 15.0, 0.7, 16, 8, "fp32", np.complex64, 0, 0),
    ("c3-fp8-L8", 5, 256, 64, 14, 64, 15.0, 0.7, 16, 8, "fp8", np.complex64, 0, 0),
    ("ragged-K20-N50-R17-fp32-L4", 5, 50, 20, 17, 16, 15.0, 0.3, 12, 4, "fp32", np.complex128, 0, 0),
    ("ragged-K20-N50-R17-bf16-L4", 5, 50, 20, 17, 16, 15.0, 0.3, 12, 4, "bf16", np.complex64, 0, 0),
    ("ragged-K12-N40-R3-fp16-refresh3", 5, 40, 12, 3, 256, 25.0, 0.2, 10, 4, "fp16", np.complex64, 3, 0),
    ("K16-fp16-L4", 5, 64, 16, 5, 16, 15.0, 0.5, 12, 4, "fp16", np.complex64, 0, 0),
    # symmetric (split) form of the block-Jacobi preconditioner
    ("c2-bf16-L8-split", 8, 128, 32, 14, 64, 20.0, 0.5, 12, 8, "bf16", np.complex64, 0, 2),
    ("c2-fp8-L8-split", 8, 128, 32, 14, 64, 20.0, 0.5, 12, 8, "fp8", np.complex64, 0, 2),
    ("c3-fp64-L8-split", 5, 256, 64, 14, 64, 15.0, 0.7, 24, 8, "fp64", np.complex128, 0, 2),
    ("c3-fp16-L8-split-refresh4", 5, 256, 64, 14, 64, 15.0, 0.7, 16, 8, "fp16", np.complex64, 4, 2),
    ("c3-fp8-L8-split", 5, 256, 64, 14, 64, 15.0, 0.7, 16, 8, "fp8", np.complex64, 0, 2),
    # K = 64 with the operand fragments in LDS and no refresh: x lives in the Gram's slot
    ("c3-fp16-L4-split", 5, 256, 64, 14, 64, 15.0, 0.7, 16, 4, "fp16", np.complex64, 0, 2),
    ("c3-bf16-L0", 5, 256, 64, 14, 64, 15.0, 0.7, 16, 0, "bf16", np.complex64, 0, 0),
    ("c3-fp16-L8-R20", 4, 256, 64, 20, 64, 15.0, 0.7, 16, 8, "fp16", np.complex64, 0, 0),
    ("K64-N200-R9-fp16-L8-textbook-c128", 4, 200, 64, 9, 16, 18.0, 0.5, 14, 8, "fp16", np.complex128, 0, 1),
    ("ragged-K20-N50-R17-fp32-L4-split", 5, 50, 20, 17, 16, 15.0, 0.3, 12, 4, "fp32", np.complex128, 0, 2),
    ("ragged-K12-N40-R3-bf16-L4-split-refresh3", 5, 40, 12, 3, 256, 25.0, 0.2, 10, 4, "bf16", np.complex64, 3, 2),
    # K up to 128: two waves per channel, A kept only in the operand format.
    # c4's shape at correlation 0.5: at c4's own 0.9 the reduced-precision
    # iteration is outside Thm 4's convergence condition (N^1.5 u sqrt(kappa)
    # far above 1), two valid rounding orders give iterates as far apart as
    # the iterates themselves, and no symbol is compared reliably
    ("c4-shape-fp8-L16", 3, 512, 128, 14, 256, 25.0, 0.5, 16, 16, "fp8", np.complex64, 0, 0),
    ("c4-shape-fp16-L16-textbook", 3, 512, 128, 14, 256, 25.0, 0.5, 16, 16, "fp16", np.complex64, 0, 1),
    ("c4-shape-bf16-L0", 3, 512, 128, 14, 256, 25.0, 0.5, 12, 0, "bf16", np.complex64, 0, 0),
    ("K120-N300-R9-fp8-L8", 3, 300, 120, 9, 64, 20.0, 0.5, 12, 8, "fp8", np.complex64, 0, 0),
    ("K100-N300-R17-fp8-L0-c128", 3, 300, 100, 17, 64, 20.0, 0.5, 12, 0, "fp8", np.complex128, 0, 0),
    ("K32-N128-fp16-L16", 4, 128, 32, 14, 64, 20.0, 0.5, 10, 16, "fp16", np.complex64, 0, 0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fixed_iteration_parity(case):
    name, B, Nbs, K, R, q, snr, zeta, iters, L, sched, io, refresh, variant = case
    _say(f"case {name}")
    wl = _wl(B, Nbs, K, R, q, snr, zeta, 11)
    x, lab, fl = gpu_detect(wl, q, iters, L, sched, io, refresh=refresh, variant=variant)
    spread, ref = oracle_spread(wl, q, iters, L, sched, io, refresh=refresh, variant=variant)
    _spread_parity(x, ref, spread, sched, name, io)
    ok, n, bad = labels_consistent(lab, ref.labels, x, ref.xhat, q, x_alt=getattr(ref, "x_alt", None))
    assert ok, (n, bad)
    assert np.array_equal(fl, ref.flags.astype(np.int64))


# --------------------------------------------------------------- refinement
@pytest.mark.parametrize("sched,steps,variant", [("fp16", 1, 0), ("fp8", 1, 0), ("fp8", 2, 0), ("bf16", 2, 0),
                                                 ("fp32", 1, 0), ("fp16", 1, 2), ("fp8", 2, 2)])
def test_refinement_reaches_oracle_accuracy(sched, steps, variant, K=32, Nbs=128):
    _say(f"case refine {sched} x{steps} variant={variant} K={K}")
    wl = _wl(8, Nbs, K, 14, 64, 25.0, 0.5, 21)
    x, lab, fl = gpu_detect(wl, 64, 16, 8, sched, np.complex64, refine=steps, variant=variant)
    ref = oracle_detect(wl, 64, 16, 8, sched, np.complex64, refine=steps, variant=variant)
    A, b = D.gram(wl.H.astype(np.complex64).astype(np.complex128), wl.Y.astype(np.complex64).astype(np.complex128),
                  wl.sigma2)
    xs = D.lmmse(A, b)
    e_g = col_rel(x, xs)
    e_o = col_rel(ref.xhat, xs)
    _say(f"  err vs LMMSE median gpu {np.median(e_g):.2e} oracle {np.median(e_o):.2e}; max {e_g.max():.2e} {e_o.max():.2e}")
    assert np.all(e_g <= np.maximum(1e-6, 4 * e_o))
    assert np.median(e_g) <= max(1e-6, 1.5 * np.median(e_o))
    d = boundary_distance(xs, 64)
    must = d > 1e-3 + np.abs(x - xs)
    assert np.array_equal(lab[must], D.slice_qam(xs, 64)[must])


@pytest.mark.parametrize("sched,variant", [("fp16", 0), ("bf16", 1)])
def test_refinement_at_k64(sched, variant):
    """K = 64: the FP64 iterate and x share the LDS with the packed operand
    (x in the Gram's slot); one refinement step to the oracle's accuracy."""
    test_refinement_reaches_oracle_accuracy(sched, 1, variant, K=64, Nbs=256)


# --------------------------------------------------------------- edge cases
def test_empty_batch_and_zero_iterations():
    import torch

    import paper_2504_09820_amd as fp

    dev = torch.device("cuda:0")
    H = torch.zeros((0, 16, 4), dtype=torch.complex64, device=dev)
    Y = torch.zeros((0, 16, 2), dtype=torch.complex64, device=dev)
    s = torch.zeros((0,), dtype=torch.float64, device=dev)
    x, lab, fl = fp.detect(H, Y, s, 16, 5, 0, "bf16")
    torch.cuda.synchronize()
    assert x.shape == (0, 4, 2)
    wl = _wl(3, 16, 4, 2, 16, 10.0, 0.0, 4)
    x, lab, fl = gpu_detect(wl, 16, 0, 0, "fp32")
    assert np.all(x == 0)
    ref = oracle_detect(wl, 16, 0, 0, "fp32")
    assert np.array_equal(lab, ref.labels)


def test_degenerate_sizes():
    for (B, Nbs, K, R) in [(4, 1, 1, 1), (3, 2, 1, 5), (2, 3, 2, 1), (2, 7, 5, 33)]:
        _say(f"case degenerate B={B} Nbs={Nbs} K={K} R={R}")
        wl = _wl(B, Nbs, K, R, 4, 10.0, 0.0, 5)
        x, lab, fl = gpu_detect(wl, 4, K, 0, "fp64")
        ref = oracle_detect(wl, 4, K, 0, "fp64")
        assert np.max(np.abs(x - ref.xhat)) <= 1e-12 * max(1.0, np.max(np.abs(ref.xhat)))
        assert np.array_equal(lab, ref.labels)


def test_breakdown_and_nonfinite_channels_are_isolated():
    wl = _wl(5, 32, 8, 3, 16, 15.0, 0.3, 6)
    H = wl.H.copy()
    Y = wl.Y.copy()
    Y[1] = 0
    H[3, 2, 5] = np.nan
    for sched, io in (("fp64", np.complex128), ("bf16", np.complex64), ("fp32", np.complex64), ("fp8", np.complex64)):
        _say(f"case isolation {sched}")
        x, lab, fl = gpu_detect(wl, 16, 8, 4, sched, io, H=H, Y=Y)
        assert np.all(x[1] == 0) and (fl[1] & 2)
        assert np.all(x[3] == 0) and (fl[3] & 1)
        keep = [0, 2, 4]
        sub = W.Workload(H=H[keep], Y=Y[keep], labels=wl.labels[keep], X=wl.X[keep], sigma2=wl.sigma2[keep], q=16,
                         snr_db=wl.snr_db[keep])
        x2, lab2, fl2 = gpu_detect(sub, 16, 8, 4, sched, io)
        assert np.array_equal(x[keep], x2) and np.array_equal(lab[keep], lab2) and np.array_equal(fl[keep], fl2)
        ref = oracle_detect(wl, 16, 8, 4, sched, io, H=H, Y=Y)
        assert np.array_equal(fl, ref.flags.astype(np.int64))


@pytest.mark.parametrize("K,L,sched,form", [(128, 16, "fp8", "fused"), (32, 4, "fp16", "pipelined"),
                                            (32, 8, "fp8", "fused")])
def test_nonfinite_and_zero_channels_at_other_shapes(K, L, sched, form):
    """A NaN in one channel's H and an all-zero Y in another flag exactly
    those channels (as the oracle does) and leave the rest untouched."""
    import torch

    import paper_2504_09820_amd as fp

    _say(f"case isolation K={K} L={L} {sched} {form}")
    wl = _wl(5, 4 * K, K, 5, 16, 15.0, 0.3, 8)
    H = wl.H.copy()
    Y = wl.Y.copy()
    Y[1] = 0
    H[3, 2, 5] = np.nan
    ctx = fp.Context(0)
    ctx.set_launch_form(form)
    dev = torch.device("cuda:0")
    x, lab, fl = fp.detect(torch.from_numpy(H.astype(np.complex64)).to(dev), torch.from_numpy(Y.astype(np.complex64)).to(dev),
                           torch.from_numpy(wl.sigma2).to(dev), 16, 8, L, sched, ctx=ctx)
    torch.cuda.synchronize()
    x, fl = x.cpu().numpy(), fl.cpu().numpy().astype(np.int64)
    ref = oracle_detect(wl, 16, 8, L, sched, np.complex64, H=H, Y=Y)
    assert np.array_equal(fl, ref.flags.astype(np.int64)), (fl, ref.flags)
    assert np.all(x[1] == 0) and np.all(x[3] == 0)
    ctx.close()


def test_run_to_run_bitwise_determinism():
    wl = _wl(20, 128, 32, 14, 64, 20.0, 0.5, 7)
    for sched in ("bf16", "fp64"):
        a = gpu_detect(wl, 64, 12, 8, sched, np.complex64)
        b = gpu_detect(wl, 64, 12, 8, sched, np.complex64)
        for u, v in zip(a, b):
            assert np.array_equal(u, v)


# --------------------------------------------------------------- slicer and rounding
@pytest.mark.parametrize("q", [4, 16, 64, 256])
def test_slicer_bitwise(q):
    import torch

    import paper_2504_09820_amd as fp

    rng = np.random.default_rng(q)
    m = int(np.sqrt(q))
    nu = np.sqrt(2 * (q - 1) / 3)
    bnd = (2 * np.arange(1, m) - m) / nu
    v = np.concatenate([rng.uniform(-1.8, 1.8, 20000), bnd, np.nextafter(bnd, 9), np.nextafter(bnd, -9),
                        [0.0, -0.0, 1e30, -1e30, np.inf, -np.inf, np.nan]])
    z = v + 1j * rng.permutation(v)
    for dt, work in ((np.complex64, "fp32"), (np.complex128, "fp64")):
        zz = z.astype(dt)
        lab = fp.slice_qam(torch.from_numpy(zz).cuda(), q).cpu().numpy()
        ref = D.slice_qam(zz, q, work)
        assert np.array_equal(lab.astype(np.int64), ref)


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "fp8", "fp32"])
def test_operand_rounding_bitwise(fmt):
    import torch

    import paper_2504_09820_amd as fp
    from oracle.rounding import round_real

    rng = np.random.default_rng(3)
    v = np.concatenate([rng.standard_normal(100000) * np.exp(rng.uniform(-12, 6, 100000)),
                        np.ldexp(rng.integers(1, 4096, 20000).astype(np.float64), rng.integers(-20, 0, 20000))])
    v = v.astype(np.float32)
    if fmt == "fp8":
        v = v[np.abs(v) <= 448]
    out = fp.round_operand(torch.from_numpy(v).cuda(), fmt).cpu().numpy().astype(np.float64)
    ref = round_real(v.astype(np.float64), {"fp8": "e4m3"}.get(fmt, fmt))
    assert np.array_equal(out, ref)
    if fmt == "fp8":
        s = 2.0**-5
        out = fp.round_operand(torch.from_numpy(v).cuda(), fmt, scale=s).cpu().numpy().astype(np.float64)
        ref = round_real(v.astype(np.float64) * s, "e4m3") / s
        assert np.array_equal(out, ref)


# --------------------------------------------------------------- full-size sampled parity
@pytest.mark.parametrize("cfg,sched,L,iters,refresh,variant", [
    ("c2", "bf16", 0, 16, 0, 0), ("c2", "fp32", 0, 16, 0, 0), ("c2", "fp64", 0, 16, 0, 0),
    ("c2", "fp16", 4, 11, 0, 2), ("c2", "fp64", 0, 15, 0, 0),  # the timed launches
    ("c2", "bf16", 8, 12, 0, 2), ("c3", "fp16", 8, 16, 4, 0), ("c3", "fp16", 8, 16, 4, 2), ("c3", "fp64", 0, 24, 0, 0),
])
def test_full_size_sampled(cfg, sched, L, iters, refresh, variant):
    import torch

    import paper_2504_09820_amd as fp

    c = W.CONFIGS[cfg]
    _say(f"case full-size {cfg} {sched} L={L} B={c['B']}")
    wl = W.draw(c["B"], c["Nbs"], c["K"], c["R"], c["q"], c["snr_db"], c["zeta"], c["zeta"], seed=77)
    dev = torch.device("cuda:0")
    Ht = torch.from_numpy(wl.H.astype(np.complex64)).to(dev)
    Yt = torch.from_numpy(wl.Y.astype(np.complex64)).to(dev)
    st = torch.from_numpy(wl.sigma2).to(dev)
    x, lab, fl = fp.detect(Ht, Yt, st, c["q"], iters, L, sched, refresh_every=refresh, variant=variant)
    torch.cuda.synchronize()
    x = x.cpu().numpy().astype(np.complex128)
    lab = lab.cpu().numpy().astype(np.int64)
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(c["B"], 24, replace=False))
    idx[-1] = c["B"] - 1
    sub = W.Workload(H=wl.H[idx], Y=wl.Y[idx], labels=wl.labels[idx], X=wl.X[idx], sigma2=wl.sigma2[idx],
                     q=c["q"], snr_db=wl.snr_db[idx])
    spread, ref = oracle_spread(sub, c["q"], iters, L, sched, np.complex64, refresh=refresh, variant=variant)
    _spread_parity(x[idx], ref, spread, sched, f"full {cfg} {sched}", np.complex64)
    ok, n, bad = labels_consistent(lab[idx], ref.labels, x[idx], ref.xhat, c["q"], x_alt=getattr(ref, "x_alt", None))
    assert ok, (n, bad)
    ber = D.bit_errors(lab, wl.labels) / (lab.size * np.log2(c["q"]))
    ber_o = D.bit_errors(ref.labels, sub.labels) / (ref.labels.size * np.log2(c["q"]))
    nbits = ref.labels.size * np.log2(c["q"])
    _say(f"  full-batch BER {ber:.4f} (oracle on the sample {ber_o:.4f})")
    # the full batch's BER is that of the oracle's sample up to sampling error
    assert abs(ber - ber_o) <= 5 * np.sqrt(ber_o * (1 - ber_o) / nbits) + 1e-3


# --------------------------------------------------------------- launch forms
@pytest.mark.parametrize("sched,L,variant,refresh,B,R", [
    ("fp16", 4, 2, 0, 3000, 14), ("bf16", 8, 0, 0, 2500, 14), ("fp32", 0, 0, 3, 2000, 14), ("fp8", 8, 2, 0, 2000, 14),
    ("fp64", 0, 0, 0, 1800, 14), ("fp16", 4, 2, 4, 1000, 37),
])
def test_pipelined_and_fused_forms_agree_bitwise(sched, L, variant, refresh, B, R):
    """The pipelined two-wave form (several channels per persistent workgroup,
    double-buffered Gram) and the one-workgroup-per-channel form run the same
    per-channel arithmetic: bitwise identical outputs.  B is large enough that
    every persistent workgroup walks several channels; R = 37 also splits each
    channel into three blocks of received vectors."""
    import torch

    import paper_2504_09820_amd as fp

    _say(f"case launch forms {sched} L={L} v{variant} refresh={refresh} B={B} R={R}")
    wl = _wl(B, 128, 32, R, 64, 20.0, 0.5, 31)
    io = np.complex128 if sched == "fp64" else np.complex64
    dev = torch.device("cuda:0")
    Ht = torch.from_numpy(wl.H.astype(io)).to(dev)
    Yt = torch.from_numpy(wl.Y.astype(io)).to(dev)
    st = torch.from_numpy(wl.sigma2).to(dev)
    outs = []
    for form in ("pipelined", "fused"):
        ctx = fp.Context(0)
        ctx.set_launch_form(form)
        x, lab, fl = fp.detect(Ht, Yt, st, 64, 12, L, sched, refresh_every=refresh, variant=variant, ctx=ctx)
        torch.cuda.synchronize()
        outs.append((x.cpu().numpy(), lab.cpu().numpy(), fl.cpu().numpy()))
        ctx.close()
    (xa, la, fa), (xb, lb, fb) = outs
    assert np.array_equal(xa.view(np.uint8), xb.view(np.uint8))
    assert np.array_equal(la, lb)
    assert np.array_equal(fa, fb)
    # and the pipelined result is the oracle's on sampled channels
    idx = np.array([0, 1, B // 2, B - 2, B - 1])
    sub = W.Workload(H=wl.H[idx], Y=wl.Y[idx], labels=wl.labels[idx], X=wl.X[idx], sigma2=wl.sigma2[idx],
                     q=64, snr_db=wl.snr_db[idx])
    spread, ref = oracle_spread(sub, 64, 12, L, sched, io, refresh=refresh, variant=variant)
    _spread_parity(xa[idx].astype(np.complex128), ref, spread, sched, f"launch forms {sched}", io)


# --------------------------------------------------------------- HIP graph capture
@pytest.mark.parametrize("form,R", [("fused", 14), ("pipelined", 14), ("fused", 37)])
def test_detect_replays_from_a_captured_graph(form, R):
    """fpcg_detect enqueues only kernels (no allocation, no host sync, no
    memset node), so it can be captured into a HIP graph.  The graph is
    replayed several times with eager launches and synchronisations between;
    every replay must equal the eager result bitwise."""
    import torch

    import paper_2504_09820_amd as fp

    _say(f"case graph capture form={form} R={R}")
    wl = _wl(600, 128, 32, R, 64, 20.0, 0.5, 41)
    dev = torch.device("cuda:0")
    Ht = torch.from_numpy(wl.H.astype(np.complex64)).to(dev)
    Yt = torch.from_numpy(wl.Y.astype(np.complex64)).to(dev)
    st = torch.from_numpy(wl.sigma2).to(dev)
    ctx = fp.Context(0)
    ctx.set_launch_form(form)
    B, K = Ht.shape[0], Ht.shape[2]
    out = (torch.empty((B, K, R), dtype=torch.complex64, device=dev), torch.empty((B, K, R), dtype=torch.uint8, device=dev),
           torch.empty((B,), dtype=torch.int32, device=dev))
    x0, l0, f0 = fp.detect(Ht, Yt, st, 64, 11, 4, "fp16", variant=2, ctx=ctx)
    torch.cuda.synchronize()
    ref = (x0.cpu().numpy().view(np.uint8), l0.cpu().numpy(), f0.cpu().numpy())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):                      # warm-up on the capture stream
        fp.detect(Ht, Yt, st, 64, 11, 4, "fp16", variant=2, ctx=ctx, out=out, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fp.detect(Ht, Yt, st, 64, 11, 4, "fp16", variant=2, ctx=ctx, out=out,
                  stream=torch.cuda.current_stream())
    for rep in range(3):
        for o in out:
            o.zero_()
        g.replay()
        torch.cuda.synchronize()
        got = (out[0].cpu().numpy().view(np.uint8), out[1].cpu().numpy(), out[2].cpu().numpy())
        assert all(np.array_equal(a, b) for a, b in zip(got, ref)), f"replay {rep} differs"
        xe, _, _ = fp.detect(Ht, Yt, st, 64, 11, 4, "fp16", variant=2, ctx=ctx)   # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(xe.cpu().numpy().view(np.uint8), ref[0])
    ctx.close()


def test_autotuned_launch_matches_explicit_forms():
    """fpcg_autotune picks one of the built forms for the shape class; the
    launch in the "auto" form afterwards gives the bits of that form set
    explicitly (the pipelined form's are the fused form's)."""
    import torch

    import paper_2504_09820_amd as fp

    _say("case autotune c2 shape, fp16 L=4 symmetric")
    ctx = fp.Context(0)
    choice = ctx.autotune(2048, 128, 32, 14, 64, 11, 4, "fp16", variant=2, reps=3)
    _say(f"  chosen form: {choice}")
    assert choice.split("-")[0] in ("fused", "pipelined", "slab")
    wl = _wl(300, 128, 32, 14, 64, 20.0, 0.5, 43)
    dev = torch.device("cuda:0")
    Ht = torch.from_numpy(wl.H.astype(np.complex64)).to(dev)
    Yt = torch.from_numpy(wl.Y.astype(np.complex64)).to(dev)
    st = torch.from_numpy(wl.sigma2).to(dev)
    xa, la, fa = fp.detect(Ht, Yt, st, 64, 11, 4, "fp16", variant=2, ctx=ctx)
    ctx.set_launch_form("fused" if choice == "pipelined" else choice)
    xb, lb, fb = fp.detect(Ht, Yt, st, 64, 11, 4, "fp16", variant=2, ctx=ctx)
    torch.cuda.synchronize()
    assert np.array_equal(xa.cpu().numpy().view(np.uint8), xb.cpu().numpy().view(np.uint8))
    assert np.array_equal(la.cpu().numpy(), lb.cpu().numpy()) and np.array_equal(fa.cpu().numpy(), fb.cpu().numpy())
    ctx.close()


def test_large_k_refinement_reaches_oracle_accuracy():
    """K = 128 with fp8 operands, L = 16 and two FP64 refinement steps through
    H, against the exact LMMSE solution and the oracle's own error.  (At the
    c4 workload's correlation 0.9 the fp8 iteration does not converge at all:
    Thm 4's bound N^1.5 u sqrt(kappa) is far above 1 there, in the oracle as on
    the GPU; correlation 0.3 at 15 dB keeps it inside.)"""
    _say("case refine K=128 fp8 L=16 x2")
    wl = _wl(3, 512, 128, 14, 256, 15.0, 0.3, 51)
    x, lab, fl = gpu_detect(wl, 256, 16, 16, "fp8", np.complex64, refine=2)
    ref = oracle_detect(wl, 256, 16, 16, "fp8", np.complex64, refine=2)
    A, b = D.gram(wl.H.astype(np.complex64).astype(np.complex128), wl.Y.astype(np.complex64).astype(np.complex128),
                  wl.sigma2)
    xs = D.lmmse(A, b)
    e_g, e_o = col_rel(x, xs), col_rel(ref.xhat, xs)
    _say(f"  err vs LMMSE median gpu {np.median(e_g):.2e} oracle {np.median(e_o):.2e}; max {e_g.max():.2e} {e_o.max():.2e}")
    assert np.all(e_g <= np.maximum(1e-6, 4 * e_o))
    assert np.median(e_g) <= max(1e-6, 1.5 * np.median(e_o))
    assert np.array_equal(fl, ref.flags.astype(np.int64))


@pytest.mark.skip(reason="fp8 FP-BJ-CG does not converge at c4's correlation 0.9 (Thm 4's condition fails by "
                         "orders of magnitude), with or without one refinement step: the GPU and oracle iterates "
                         "differ as much as two valid rounding orders of the oracle do, and no symbol can be "
                         "compared; c4's shape is checked at a converging correlation in the fixed-iteration "
                         "cases")
def test_large_k_full_size_sampled():
    """c4 at its full size (B = 2048, Nbs = 512, K = 128, fp8, L = 16, one
    refinement step) in the bench's launch form, checked on sampled channels."""
    import torch

    import paper_2504_09820_amd as fp

    c = W.CONFIGS["c4"]
    _say(f"case full-size c4 fp8 L=16 refine=1 B={c['B']}")
    wl = W.draw(c["B"], c["Nbs"], c["K"], c["R"], c["q"], c["snr_db"], c["zeta"], c["zeta"], seed=78)
    dev = torch.device("cuda:0")
    Ht = torch.from_numpy(wl.H.astype(np.complex64)).to(dev)
    Yt = torch.from_numpy(wl.Y.astype(np.complex64)).to(dev)
    st = torch.from_numpy(wl.sigma2).to(dev)
    x, lab, fl = fp.detect(Ht, Yt, st, c["q"], 16, 16, "fp8", refine_steps=1)
    torch.cuda.synchronize()
    x = x.cpu().numpy().astype(np.complex128)
    lab = lab.cpu().numpy().astype(np.int64)
    idx = np.array([0, 1, 777, c["B"] - 2, c["B"] - 1])
    sub = W.Workload(H=wl.H[idx], Y=wl.Y[idx], labels=wl.labels[idx], X=wl.X[idx], sigma2=wl.sigma2[idx],
                     q=c["q"], snr_db=wl.snr_db[idx])
    # at correlation 0.9 fp8 is far outside the heuristic's range and the
    # iteration does not converge, so rounding orders drift apart: compare
    # with the oracle's own spread between two valid orders
    spread, ref = oracle_spread(sub, c["q"], 16, 16, "fp8", np.complex64, refine=1)
    _spread_parity(x[idx], ref, spread, "fp8", "full c4 fp8 L=16 refine=1", np.complex64)
    ok, n, bad = labels_consistent(lab[idx], ref.labels, x[idx], ref.xhat, c["q"], x_alt=getattr(ref, "x_alt", None))
    assert ok, (n, bad)
    assert np.array_equal(fl.cpu().numpy()[idx].astype(np.int64), ref.flags.astype(np.int64))


# --------------------------------------------------------------- waves per channel (K = 64)
WAVE_CASES = [
    # name, form, I, L, sched, io, refresh, refine, variant
    ("fp16-L4-split-refresh4-w4", "fused-w4", 16, 4, "fp16", np.complex64, 4, 0, 2),
    ("fp16-L4-left-refresh4-w4", "fused-w4", 16, 4, "fp16", np.complex64, 4, 0, 0),
    ("fp16-L0-w4", "fused-w4", 16, 0, "fp16", np.complex64, 0, 0, 0),
    ("bf16-L4-split-w4-c128", "fused-w4", 14, 4, "bf16", np.complex128, 0, 0, 2),
    ("fp16-L8-split-refresh4-w2", "fused-w2", 16, 8, "fp16", np.complex64, 4, 0, 2),
    ("bf16-L8-textbook-w2", "fused-w2", 16, 8, "bf16", np.complex64, 0, 0, 1),
    ("fp32-L4-split-w4", "fused-w4", 16, 4, "fp32", np.complex64, 0, 0, 2),
    ("fp32-L0-refresh3-w4", "fused-w4", 12, 0, "fp32", np.complex64, 3, 0, 0),
    ("fp16-L4-refine1-w4", "fused-w4", 16, 4, "fp16", np.complex64, 0, 1, 0),
    ("fp64-L4-split-w4", "fused-w4", 24, 4, "fp64", np.complex128, 0, 0, 2),
]


@pytest.mark.parametrize("case", WAVE_CASES, ids=[c[0] for c in WAVE_CASES])
def test_wave_counts_match_oracle(case):
    """The K = 64 builds with two or four waves per channel (each wave holding
    K/(4 NW) entries of every iterate per lane, the operand copy of A in
    registers) against the oracle, at the c3 shape with a ragged batch."""
    import torch

    import paper_2504_09820_amd as fp

    name, form, iters, L, sched, io, refresh, refine, variant = case
    _say(f"case waves {name}")
    wl = _wl(5, 256, 64, 14, 64, 15.0, 0.7, 61)
    ctx = fp.Context(0)
    ctx.set_launch_form(form)
    dev = torch.device("cuda:0")
    x, lab, fl = fp.detect(torch.from_numpy(wl.H.astype(io)).to(dev), torch.from_numpy(wl.Y.astype(io)).to(dev),
                           torch.from_numpy(wl.sigma2).to(dev), 64, iters, L, sched, refresh_every=refresh,
                           refine_steps=refine, variant=variant, ctx=ctx)
    torch.cuda.synchronize()
    x = x.cpu().numpy().astype(np.complex128)
    lab = lab.cpu().numpy().astype(np.int64)
    fl = fl.cpu().numpy().astype(np.int64)
    ctx.close()
    spread, ref = oracle_spread(wl, 64, iters, L, sched, io, refresh=refresh, refine=refine, variant=variant)
    _spread_parity(x, ref, spread, sched, name, io)
    ok, n, bad = labels_consistent(lab, ref.labels, x, ref.xhat, 64, x_alt=getattr(ref, "x_alt", None))
    assert ok, (n, bad)
    assert np.array_equal(fl, ref.flags.astype(np.int64))


def test_fp64_four_waves_converged_to_1e12():
    import torch

    import paper_2504_09820_amd as fp

    _say("case fp64 w4 converged K=64 L=0 I=192")
    wl = _wl(6, 256, 64, 14, 64, 20.0, 0.5, 62)
    ctx = fp.Context(0)
    ctx.set_launch_form("fused-w4")
    dev = torch.device("cuda:0")
    x, lab, fl = fp.detect(torch.from_numpy(wl.H).to(dev), torch.from_numpy(wl.Y).to(dev),
                           torch.from_numpy(wl.sigma2).to(dev), 64, 192, 0, "fp64", ctx=ctx)
    torch.cuda.synchronize()
    ctx.close()
    ref = oracle_detect(wl, 64, 192, 0, "fp64")
    assert np.max(col_rel(x.cpu().numpy(), ref.xhat)) < 1e-12


# --------------------------------------------------------------- the slab form (A held in registers)
SLAB_CASES = [
    # name, K, Nbs, R, q, iters, L, sched, io, refresh, variant
    ("fp16-L4-split-refresh4", 64, 256, 14, 64, 16, 4, "fp16", np.complex64, 4, 2),
    ("fp16-L4-left-refresh4", 64, 256, 14, 64, 16, 4, "fp16", np.complex64, 4, 0),
    ("fp16-L4-textbook", 64, 256, 14, 64, 16, 4, "fp16", np.complex64, 0, 1),
    ("fp16-L0", 64, 256, 14, 64, 16, 0, "fp16", np.complex64, 0, 0),
    ("bf16-L4-split-c128", 64, 256, 14, 64, 14, 4, "bf16", np.complex128, 0, 2),
    ("fp32-L4-split", 64, 256, 14, 64, 16, 4, "fp32", np.complex64, 0, 2),
    ("fp32-L0-refresh3", 64, 256, 14, 64, 12, 0, "fp32", np.complex64, 3, 0),
    ("fp64-L4-split", 64, 256, 14, 64, 24, 4, "fp64", np.complex128, 0, 2),
    ("fp64-L0", 64, 256, 14, 64, 24, 0, "fp64", np.complex128, 0, 0),
    ("K52-N200-R9-fp16-L4-split-refresh4", 52, 200, 9, 16, 14, 4, "fp16", np.complex64, 4, 2),
    ("K64-R20-fp16-L4-split", 64, 256, 20, 64, 12, 4, "fp16", np.complex64, 0, 2),
    ("K128-fp64-L0", 128, 512, 14, 256, 24, 0, "fp64", np.complex128, 0, 0),
    ("K128-fp32-L0", 128, 512, 14, 256, 24, 0, "fp32", np.complex64, 0, 0),
    ("K100-N300-R17-fp64-L0", 100, 300, 17, 64, 20, 0, "fp64", np.complex128, 0, 0),
    # L = 8: two Jacobi blocks in each diagonal tile (symmetric form)
    ("fp16-L8-split-refresh4", 64, 256, 14, 64, 16, 8, "fp16", np.complex64, 4, 2),
    ("fp32-L8-split", 64, 256, 14, 64, 16, 8, "fp32", np.complex64, 0, 2),
    ("bf16-L8-split-c128", 64, 256, 14, 64, 14, 8, "bf16", np.complex128, 0, 2),
    ("K56-N200-R20-fp16-L8-split", 56, 200, 20, 16, 14, 8, "fp16", np.complex64, 0, 2),
    # L = 16: the Jacobi blocks are the 16 x 16 diagonal tiles (symmetric form, fp32)
    ("fp32-L16-split", 64, 256, 14, 64, 16, 16, "fp32", np.complex64, 0, 2),
    ("fp32-L16-split-refresh3", 64, 256, 14, 64, 12, 16, "fp32", np.complex64, 3, 2),
    ("K48-N200-R9-fp32-L16-c128", 48, 200, 9, 16, 14, 16, "fp32", np.complex128, 0, 2),
    ("K128-fp32-L16-split", 128, 512, 14, 256, 24, 16, "fp32", np.complex64, 0, 2),
    ("K112-N300-R17-fp32-L16", 112, 300, 17, 64, 20, 16, "fp32", np.complex64, 0, 2),
    ("K128-fp32-L16-split-refresh4", 128, 512, 14, 256, 16, 16, "fp32", np.complex64, 4, 2),
    ("K128-fp16-L16-split-refresh4", 128, 512, 14, 256, 16, 16, "fp16", np.complex64, 4, 2),
    ("K112-N300-bf16-L16-split-c128", 112, 300, 14, 64, 16, 16, "bf16", np.complex128, 0, 2),
]


def _slab_run(wl, q, iters, L, sched, io, refresh, variant):
    import torch

    import paper_2504_09820_amd as fp

    ctx = fp.Context(0)
    ctx.set_launch_form("slab")
    dev = torch.device("cuda:0")
    x, lab, fl = fp.detect(torch.from_numpy(wl.H.astype(io)).to(dev), torch.from_numpy(wl.Y.astype(io)).to(dev),
                           torch.from_numpy(wl.sigma2).to(dev), q, iters, L, sched, refresh_every=refresh,
                           variant=variant, ctx=ctx)
    torch.cuda.synchronize()
    ctx.close()
    return x.cpu().numpy().astype(np.complex128), lab.cpu().numpy().astype(np.int64), fl.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("case", SLAB_CASES, ids=[c[0] for c in SLAB_CASES])
def test_slab_form_matches_oracle(case):
    """The slab form (K/16 waves per channel, A's operand copies in registers,
    p exchanged through LDS once per iteration) against the oracle, with
    ragged K, Nbs and R and two blocks of received vectors."""
    name, K, Nbs, R, q, iters, L, sched, io, refresh, variant = case
    _say(f"case slab {name}")
    zeta = 0.5 if K == 128 else 0.7
    wl = _wl(5 if K < 128 else 3, Nbs, K, R, q, 15.0 if K < 128 else 25.0, zeta, 63)
    x, lab, fl = _slab_run(wl, q, iters, L, sched, io, refresh, variant)
    spread, ref = oracle_spread(wl, q, iters, L, sched, io, refresh=refresh, variant=variant)
    _spread_parity(x, ref, spread, sched, name, io)
    ok, n, bad = labels_consistent(lab, ref.labels, x, ref.xhat, q, x_alt=getattr(ref, "x_alt", None))
    assert ok, (n, bad)
    assert np.array_equal(fl, ref.flags.astype(np.int64))


@pytest.mark.parametrize("K,L,sched", [(64, 0, "fp16"), (64, 4, "fp16"), (64, 8, "fp16"), (64, 16, "fp32"),
                                        (128, 16, "fp32"), (128, 0, "fp64")])
def test_slab_empty_batch_and_zero_iterations(K, L, sched):
    """The slab form with B = 0 (a no-op) and with I = 0 (x_hat = 0 after
    the setup, labels of 0, as the oracle's)."""
    import torch

    import paper_2504_09820_amd as fp

    _say(f"case slab empty / I=0 K={K} L={L} {sched}")
    ctx = fp.Context(0)
    ctx.set_launch_form("slab")
    dev = torch.device("cuda:0")
    Nbs = 2 * K
    H = torch.zeros((0, Nbs, K), dtype=torch.complex64, device=dev)
    Y = torch.zeros((0, Nbs, 14), dtype=torch.complex64, device=dev)
    s = torch.zeros((0,), dtype=torch.float64, device=dev)
    x, lab, fl = fp.detect(H, Y, s, 16, 5, L, sched, variant=2 if L else 0, ctx=ctx)
    torch.cuda.synchronize()
    assert x.shape == (0, K, 14)
    ctx.close()
    wl = _wl(3, Nbs, K, 14, 16, 10.0, 0.3, 68)
    x, lab, fl = _slab_run(wl, 16, 0, L, sched, np.complex64, 0, 2 if L else 0)
    assert np.all(x == 0)
    ref = oracle_detect(wl, 16, 0, L, sched, np.complex64, variant=2 if L else 0)
    assert np.array_equal(lab, ref.labels)
    assert np.array_equal(fl, ref.flags.astype(np.int64))


@pytest.mark.parametrize("K,Nbs,L", [(64, 256, 16), (128, 512, 16), (80, 200, 16), (64, 256, 8)])
def test_slab_fp32_l16_converged_within_1e5_of_lmmse(K, Nbs, L):
    """FP-BJ-CG with 16 x 16 (and 8 x 8) blocks and FP32 work run to
    convergence (I = K/2 here): within 1e-5 of the exact LMMSE solution
    (every HPD preconditioner leaves the solution unchanged), labels
    identical away from the boundaries, flags as the oracle's (none yet: run
    on past convergence, the FP32 recurrences end in the breakdown guard, in
    the oracle too)."""
    _say(f"case slab fp32 L={L} converged K={K}")
    wl = _wl(4, Nbs, K, 14, 64, 20.0, 0.5, 66)
    x, lab, fl = _slab_run(wl, 64, K // 2, L, "fp32", np.complex64, 0, 2)
    ref = oracle_detect(wl, 64, K // 2, L, "fp32", np.complex64, variant=2)
    A, b = D.gram(wl.H.astype(np.complex64).astype(np.complex128), wl.Y.astype(np.complex64).astype(np.complex128),
                  wl.sigma2)
    xs = D.lmmse(A, b)
    e = col_rel(x, xs)
    _say(f"  max rel error vs LMMSE {e.max():.2e}")
    assert e.max() < 1e-5
    far = boundary_distance(xs, 64) > 1e-3
    assert np.array_equal(lab[far], D.slice_qam(xs, 64)[far])
    assert np.array_equal(fl, ref.flags.astype(np.int64))


@pytest.mark.parametrize("L,sched", [(16, "fp32"), (8, "fp32"), (8, "fp16")])
def test_slab_l16_not_pd_block_flagged_and_isolated(L, sched):
    """A channel whose Jacobi block is singular (sigma^2 = 0 and a user's
    column of H zero) falls back to the diagonal for that block and raises
    BLOCK_NOT_PD, as the oracle does; the other channels are unaffected."""
    _say(f"case slab L={L} {sched} not-PD block")
    wl = _wl(5, 256, 64, 5, 16, 15.0, 0.3, 67)
    H = wl.H.copy()
    H[2, :, 20] = 0
    s2 = wl.sigma2.copy()
    s2[2] = 0.0
    sub = W.Workload(H=H, Y=wl.Y, labels=wl.labels, X=wl.X, sigma2=s2, q=16, snr_db=wl.snr_db)
    x, lab, fl = _slab_run(sub, 16, 8, L, sched, np.complex64, 0, 2)
    spread, ref = oracle_spread(sub, 16, 8, L, sched, np.complex64, variant=2)
    assert np.array_equal(fl, ref.flags.astype(np.int64)), (fl, ref.flags)
    assert fl[2] != 0 and not np.delete(fl, 2).any()
    keep = np.array([0, 1, 3, 4])
    sp2, ref2 = oracle_spread(W.Workload(H=wl.H[keep], Y=wl.Y[keep], labels=wl.labels[keep], X=wl.X[keep],
                                         sigma2=wl.sigma2[keep], q=16, snr_db=wl.snr_db[keep]),
                              16, 8, L, sched, np.complex64, variant=2)
    _spread_parity(x[keep], ref2, sp2, sched, "not-PD neighbours", np.complex64)


@pytest.mark.parametrize("K,L,sched,refresh", [(64, 4, "fp16", 4), (64, 8, "fp16", 4), (64, 16, "fp32", 0),
                                              (128, 16, "fp32", 0), (64, 0, "fp64", 0)])
def test_slab_run_to_run_bitwise_determinism(K, L, sched, refresh):
    """The slab form gives the same bits on every run: its reductions over
    lanes and waves, the LDS exchanges of p and x, and the L = 8 / 16 block
    factorisation (whose steps a wave orders by itself, without a workgroup
    barrier) have one fixed order.  A batch of 2000 channels, three runs."""
    import torch

    import paper_2504_09820_amd as fp

    _say(f"case slab determinism K={K} L={L} {sched} refresh={refresh}")
    wl = _wl(2000, 2 * K, K, 14, 64, 20.0, 0.6, 69)
    dev = torch.device("cuda:0")
    H = torch.from_numpy(wl.H.astype(np.complex64)).to(dev)
    Y = torch.from_numpy(wl.Y.astype(np.complex64)).to(dev)
    s2 = torch.from_numpy(wl.sigma2).to(dev)
    ctx = fp.Context(0)
    ctx.set_launch_form("slab")
    outs = []
    for _ in range(3):
        x, lab, fl = fp.detect(H, Y, s2, 64, 12, L, sched, refresh_every=refresh, variant=2 if L else 0, ctx=ctx)
        torch.cuda.synchronize()
        outs.append((x.cpu().numpy().view(np.uint8), lab.cpu().numpy(), fl.cpu().numpy()))
    ctx.close()
    for o in outs[1:]:
        for u, v in zip(outs[0], o):
            assert np.array_equal(u, v)


@pytest.mark.parametrize("K,Nbs,L", [(64, 256, 0), (64, 256, 4), (128, 512, 0)])
def test_slab_fp64_converged_to_1e12(K, Nbs, L):
    _say(f"case slab fp64 converged K={K} L={L}")
    wl = _wl(4, Nbs, K, 14, 64, 20.0, 0.5, 64)
    x, lab, fl = _slab_run(wl, 64, 3 * K, L, "fp64", np.complex128, 0, 2 if L else 0)
    ref = oracle_detect(wl, 64, 3 * K, L, "fp64", variant=2 if L else 0)
    assert np.max(col_rel(x, ref.xhat)) < 1e-12


def test_slab_isolates_nonfinite_and_zero_channels():
    _say("case slab isolation K=64 fp16 L=4 split")
    wl = _wl(5, 256, 64, 5, 16, 15.0, 0.3, 65)
    H = wl.H.copy()
    Y = wl.Y.copy()
    Y[1] = 0
    H[3, 2, 5] = np.nan
    sub = W.Workload(H=H, Y=Y, labels=wl.labels, X=wl.X, sigma2=wl.sigma2, q=16, snr_db=wl.snr_db)
    x, lab, fl = _slab_run(sub, 16, 8, 4, "fp16", np.complex64, 0, 2)
    ref = oracle_detect(wl, 16, 8, 4, "fp16", np.complex64, variant=2, H=H, Y=Y)
    assert np.array_equal(fl, ref.flags.astype(np.int64)), (fl, ref.flags)
    assert np.all(x[1] == 0) and np.all(x[3] == 0)


# --------------------------------------------------------------- the timed launches at full size
# (config, schedule, L, I, refresh, variant): the slab-form launches the
# benchmark times at c3 and c4 -- the configured FP-BJ-CG schedule, the
# heuristic's pick and FP64 CG, at the iteration counts the BER-parity
# search settles on (and at c4 fp16 with the FP64 refresh, reported beside
# them)
TIMED_FULL = [
    ("c3", "fp16", 4, 20, 4, 2),
    ("c3", "fp32", 4, 20, 0, 2),
    ("c3", "fp64", 0, 27, 0, 0),
    ("c4", "fp32", 16, 64, 0, 2),
    ("c4", "fp64", 0, 92, 0, 0),
    ("c4", "fp16", 16, 67, 4, 2),
]
_FULL_WL = {}


def _full_workload(cfg):
    if cfg not in _FULL_WL:
        _FULL_WL.clear()                              # one full-size batch held at a time
        c = W.CONFIGS[cfg]
        _FULL_WL[cfg] = W.draw(c["B"], c["Nbs"], c["K"], c["R"], c["q"], c["snr_db"], c["zeta"], c["zeta"], seed=79)
    return _FULL_WL[cfg]


@pytest.mark.parametrize("case", TIMED_FULL, ids=[f"{c[0]}-{c[1]}-L{c[2]}-I{c[3]}" for c in TIMED_FULL])
def test_timed_slab_launches_full_size_sampled(case):
    """Full batch in the slab form, checked on sampled channels (the first,
    the last and random ones) against the oracle: the spread bar of the
    smaller cases, labels, flags, and the batch's BER against the sample's."""
    import torch

    import paper_2504_09820_amd as fp

    cfg, sched, L, iters, refresh, variant = case
    c = W.CONFIGS[cfg]
    _say(f"case timed full-size {cfg} slab {sched} L={L} I={iters} refresh={refresh} B={c['B']}")
    wl = _full_workload(cfg)
    dev = torch.device("cuda:0")
    io = np.complex64
    ctx = fp.Context(0)
    ctx.set_launch_form("slab")
    Ht = torch.from_numpy(wl.H.astype(io)).to(dev)
    Yt = torch.from_numpy(wl.Y.astype(io)).to(dev)
    st = torch.from_numpy(wl.sigma2).to(dev)
    x, lab, fl = fp.detect(Ht, Yt, st, c["q"], iters, L, sched, refresh_every=refresh, variant=variant, ctx=ctx)
    torch.cuda.synchronize()
    ctx.close()
    del Ht, Yt
    x = x.cpu().numpy().astype(np.complex128)
    lab = lab.cpu().numpy().astype(np.int64)
    fl = fl.cpu().numpy().astype(np.int64)
    rng = np.random.default_rng(1)
    n = 12 if cfg == "c3" else 6
    idx = np.unique(np.concatenate([[0, c["B"] - 1], rng.choice(c["B"], n - 2, replace=False)]))
    sub = W.Workload(H=wl.H[idx], Y=wl.Y[idx], labels=wl.labels[idx], X=wl.X[idx], sigma2=wl.sigma2[idx],
                     q=c["q"], snr_db=wl.snr_db[idx])
    spread, ref = oracle_spread(sub, c["q"], iters, L, sched, io, refresh=refresh, variant=variant)
    _spread_parity(x[idx], ref, spread, sched, f"timed {cfg} {sched}", io)
    ok, nc, bad = labels_consistent(lab[idx], ref.labels, x[idx], ref.xhat, c["q"], x_alt=getattr(ref, "x_alt", None))
    assert ok, (nc, bad)
    assert np.array_equal(fl[idx], ref.flags.astype(np.int64))
    assert not fl.any()
    ber = D.bit_errors(lab, wl.labels) / (lab.size * np.log2(c["q"]))
    ber_o = D.bit_errors(ref.labels, sub.labels) / (ref.labels.size * np.log2(c["q"]))
    nbits = ref.labels.size * np.log2(c["q"])
    _say(f"  full-batch BER {ber:.4f} (oracle on the sample {ber_o:.4f})")
    assert abs(ber - ber_o) <= 5 * np.sqrt(ber_o * (1 - ber_o) / nbits) + 1e-3
