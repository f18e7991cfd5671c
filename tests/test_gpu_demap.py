"""Soft output through the C ABI: the detector's effective gains against the
oracle's (eq. pre_BJ block inverses of the oracle's own Gram), the max-log
demapper against the oracle's brute force over all Q points, and the two
composed after a converged FP64 detection."""
import math
import sys

import numpy as np
import pytest

import workload as W
from oracle import demap as DM
from tests.gpu_common import oracle_detect

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _demap_gpu(x, gain, q):
    import torch

    import paper_2504_09820_amd as fp

    dev = torch.device("cuda:0")
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    gt = torch.from_numpy(np.ascontiguousarray(gain.astype(np.float32))).to(dev)
    llr = fp.demap_maxlog(xt, gt, q)
    torch.cuda.synchronize()
    return llr.cpu().numpy().astype(np.float64)


def _llr_tolerance(x, gain, q, u):
    """Rounding bound of the demapper's arithmetic at unit roundoff u: each
    distance (v - mu a)^2 carries a few roundings of (|v| + mu a_max)^2, the
    difference of two and the scaling by 1 / nu^2 a few more."""
    g = np.clip(np.asarray(gain, dtype=np.float64), 0, 1)
    amax = (math.isqrt(q) - 1) / math.sqrt(2.0 * (q - 1) / 3.0)
    v = np.maximum(np.abs(x.real), np.abs(x.imag))
    with np.errstate(divide="ignore"):
        s = 1.0 / (g * (1 - g))
    return (16 * u * (v + g * amax) ** 2 * s)[..., None]


def _compare_llr(got, ref, tol, u):
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    inf = np.isinf(ref)
    assert np.array_equal(np.isinf(got), inf) and np.array_equal(np.sign(got[inf]), np.sign(ref[inf]))
    fin = ~nan & ~inf
    err = np.abs(got - ref)[fin]
    # plus the rounding of the result to the float32 output
    bound = (np.broadcast_to(tol, ref.shape) + (4 * u + 2.0**-24) * np.abs(ref))[fin]
    assert np.all(err <= bound), (err.max(), np.max(err / bound))


@pytest.mark.parametrize("io", [np.complex64, np.complex128])
@pytest.mark.parametrize("q", [4, 16, 64, 256])
def test_demap_matches_oracle(q, io):
    rng = np.random.default_rng(q + (io == np.complex128))
    B, K, R = 7, 5, 13                                    # 455 symbols: ragged against the 256-thread blocks
    x = ((rng.standard_normal((B, K, R)) + 1j * rng.standard_normal((B, K, R))) * 0.9).astype(io)
    gain = rng.uniform(0.02, 0.999, (B, K)).astype(np.float32)
    gain[0, :4] = [0.0, 1.0, -1e-7, 1.0 + 1e-7]            # no signal, zero-forcing, rounding outside [0, 1]
    gain[1, 0] = np.nan
    x[2, 0, 0] = np.nan                                   # real part NaN, imaginary 0
    x[3, 1, 2] = complex(0.3, np.inf)
    _say(f"case demap q={q} io={np.dtype(io).name} n={x.size}")
    got = _demap_gpu(x, gain, q)
    xr = x.astype(np.complex128)
    ref = DM.maxlog_llr(xr, gain.astype(np.float64)[..., None], q)
    u = 2.0**-24 if io == np.complex64 else 2.0**-53
    _compare_llr(got, ref, _llr_tolerance(xr, gain[..., None], q, u), u)


def test_demap_many_blocks_and_per_symbol_gains():
    # more symbols than one pass of the grid-stride loop covers at 65535 x 256
    import torch

    import paper_2504_09820_amd as fp

    q, n = 64, 65535 * 256 + 1001
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(7)
    x = torch.randn((n,), dtype=torch.complex64, device=dev, generator=g).reshape(1, 1, n)
    gain = torch.rand((1, 1), dtype=torch.float32, device=dev, generator=g) * 0.9 + 0.05
    llr = fp.demap_maxlog(x, gain, q)
    torch.cuda.synchronize()
    _say(f"case demap n={n}")
    # sampled symbols against the oracle, the tail included
    idx = np.concatenate([np.arange(0, 2000), np.arange(n - 3000, n), np.random.default_rng(1).integers(0, n, 4000)])
    xs = x.reshape(-1)[torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.complex128)
    gs = float(gain.item())
    ref = DM.maxlog_llr(xs, np.full(idx.size, gs), q)
    got = llr.reshape(n, 6)[torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.float64)
    _compare_llr(got, ref, _llr_tolerance(xs, np.full(idx.size, gs), q, 2.0**-24), 2.0**-24)


def _gain_gpu(wl, io, qam, iters, L, sched, variant=0):
    import torch

    import paper_2504_09820_amd as fp

    dev = torch.device("cuda:0")
    Ht = torch.from_numpy(np.ascontiguousarray(wl.H.astype(io))).to(dev)
    Yt = torch.from_numpy(np.ascontiguousarray(wl.Y.astype(io))).to(dev)
    st = torch.from_numpy(np.ascontiguousarray(wl.sigma2)).to(dev)
    B, _, K = wl.H.shape
    gain = torch.full((B, K), -7.0, dtype=torch.float32, device=dev)
    x, lab, fl = fp.detect(Ht, Yt, st, qam, iters, L, sched, variant=variant, gain=gain)
    torch.cuda.synchronize()
    return x.cpu().numpy().astype(np.complex128), gain.cpu().numpy().astype(np.float64), fl.cpu().numpy()


@pytest.mark.parametrize("K,L,variant", [(8, 0, 0), (4, 4, 0), (32, 4, 2), (32, 8, 1), (64, 8, 0)])
def test_gain_fp64_matches_oracle(K, L, variant):
    wl = W.draw(12, 4 * K, K, 3, 16, 12.0, 0.6, 0.6, seed=70 + K + L)
    _say(f"case gain fp64 K={K} L={L} v{variant}")
    _, g, fl = _gain_gpu(wl, np.complex128, 16, 2 * K, L, "fp64", variant)
    ref = oracle_detect(wl, 16, 2 * K, L, "fp64", variant=variant)
    gr = DM.effective_gain(ref.A, wl.sigma2, L)
    assert np.all(fl == 0)
    np.testing.assert_allclose(g, gr, rtol=0, atol=2.0**-24)     # FP64 gain stored as float32


@pytest.mark.parametrize("sched,K,L,variant", [("fp16", 32, 4, 2), ("fp32", 64, 8, 0), ("bf16", 32, 0, 0),
                                               ("fp16", 128, 16, 0), ("bf16", 128, 0, 0)])
def test_gain_reduced_matches_oracle(sched, K, L, variant):
    wl = W.draw(10, 2 * K if K < 128 else 256, K, 14, 64, 18.0, 0.5, 0.5, seed=80 + K + L)
    _say(f"case gain {sched} K={K} L={L} v{variant}")
    _, g, _ = _gain_gpu(wl, np.complex64, 64, 8, L, sched, variant)
    r1 = oracle_detect(wl, 64, 8, L, sched, io=np.complex64, variant=variant, accum="exact")
    r2 = oracle_detect(wl, 64, 8, L, sched, io=np.complex64, variant=variant, accum="sequential")
    g1 = DM.effective_gain(r1.A, wl.sigma2, L, "fp32")
    g2 = DM.effective_gain(r2.A, wl.sigma2, L, "fp32")
    spread = np.abs(g1 - g2).max()
    # the GPU is a third rounding order of the u_W Gram; its block inverse is
    # formed in u_W (the oracle's in FP64, rounded once)
    tol = 4 * spread + 16 * max(L, 1) * 2.0**-24
    _say(f"  gain gpu-oracle max {np.abs(g - g1).max():.2e}, oracle order spread {spread:.2e}, tol {tol:.2e}")
    assert np.all(np.abs(g - g1) <= tol)
    assert np.all((g > 0) & (g < 1))


def test_soft_output_after_converged_detection():
    wl = W.draw(16, 128, 32, 14, 64, 22.0, 0.5, 0.5, seed=91)
    _say("case soft output fp64 L=4 v2 I=96")
    x, g, fl = _gain_gpu(wl, np.complex128, 64, 96, 4, "fp64", variant=2)
    llr = _demap_gpu(x, g.astype(np.float32), 64)
    ref = oracle_detect(wl, 64, 96, 4, "fp64", variant=2)
    gr = DM.effective_gain(ref.A, wl.sigma2, 4).astype(np.float32).astype(np.float64)
    lo = DM.maxlog_llr(ref.xhat, gr[..., None], 64)
    assert np.all(fl == 0) and np.array_equal(g, gr)
    # x_hat agrees to 1e-12: the demapper's FP64 rounding plus that difference
    dx = np.abs(x - ref.xhat).max()
    amax = 7 / math.sqrt(42)
    s = 1.0 / (gr * (1 - gr))
    tol = _llr_tolerance(ref.xhat, gr[..., None], 64, 2.0**-53) + (8 * dx * (np.abs(ref.xhat) + amax) * s[..., None])[..., None]
    _compare_llr(llr, lo, tol, 2.0**-53)
    # hard decisions from the LLR signs: the unbiased estimate's nearest point
    nb = 6
    bits = (llr < 0).astype(np.int64)
    lab = sum(bits[..., t] << (nb - 1 - t) for t in range(nb))
    from oracle import detect as D
    assert np.array_equal(lab, D.slice_qam(ref.xhat / gr[..., None], 64))


def test_soft_output_full_size_sampled():
    """The bench's soft path at its full size (c2: 16384 channels, fp16, L = 4,
    symmetric form, I = 11, with gains, then the demapper): gains of sampled
    channels against the oracle's from its own Gram, and the LLRs of those
    channels against the oracle's demapping of the GPU's estimates and gains."""
    import torch

    import paper_2504_09820_amd as fp

    c = W.CONFIGS["c2"]
    B, K, R, q = c["B"], c["K"], c["R"], c["q"]
    _say(f"case soft output full size c2 B={B}")
    wl = W.draw(B, c["Nbs"], K, R, q, c["snr_db"], c["zeta"], c["zeta"], seed=78)
    dev = torch.device("cuda:0")
    Ht = torch.from_numpy(wl.H.astype(np.complex64)).to(dev)
    Yt = torch.from_numpy(wl.Y.astype(np.complex64)).to(dev)
    st = torch.from_numpy(wl.sigma2).to(dev)
    g = torch.empty((B, K), dtype=torch.float32, device=dev)
    x, _, _ = fp.detect(Ht, Yt, st, q, 11, 4, "fp16", variant=2, gain=g)
    llr = fp.demap_maxlog(x, g, q)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(2).choice(B, 24, replace=False))
    idx[-1] = B - 1
    ti = torch.from_numpy(idx).to(dev)
    xs = x[ti].cpu().numpy().astype(np.complex128)
    gs = g[ti].cpu().numpy().astype(np.float64)
    ls = llr[ti].cpu().numpy().astype(np.float64)
    sub = W.Workload(H=wl.H[idx], Y=wl.Y[idx], labels=wl.labels[idx], X=wl.X[idx], sigma2=wl.sigma2[idx],
                     q=q, snr_db=wl.snr_db[idx])
    r1 = oracle_detect(sub, q, 11, 4, "fp16", io=np.complex64, variant=2, accum="exact")
    r2 = oracle_detect(sub, q, 11, 4, "fp16", io=np.complex64, variant=2, accum="sequential")
    g1 = DM.effective_gain(r1.A, sub.sigma2, 4, "fp32")
    spread = np.abs(g1 - DM.effective_gain(r2.A, sub.sigma2, 4, "fp32")).max()
    assert np.all(np.abs(gs - g1) <= 4 * spread + 64 * 2.0**-24)
    ref = DM.maxlog_llr(xs, gs[..., None], q)
    _compare_llr(ls, ref, _llr_tolerance(xs, gs[..., None], q, 2.0**-24), 2.0**-24)


def test_gain_depends_on_the_channel_only():
    """Gains come from A alone: the same channels with R = 3 and R = 37 (three
    workgroups per channel, only the first writes gains) give bitwise equal
    gains; an indexed launch writes them for its channels only."""
    import torch

    import paper_2504_09820_amd as fp

    B, K = 20, 32
    wl3 = W.draw(B, 128, K, 3, 64, 18.0, 0.5, 0.5, seed=93)
    wl37 = W.draw(B, 128, K, 37, 64, 18.0, 0.5, 0.5, seed=94)
    _say("case gain vs R and indexed launch")
    dev = torch.device("cuda:0")
    Ht = torch.from_numpy(wl3.H.astype(np.complex64)).to(dev)
    st = torch.from_numpy(wl3.sigma2).to(dev)
    gains = []
    for wl in (wl3, wl37):
        Yt = torch.from_numpy(wl.Y.astype(np.complex64)).to(dev)
        g = torch.full((B, K), -7.0, dtype=torch.float32, device=dev)
        fp.detect(Ht, Yt, st, 64, 11, 4, "fp16", variant=2, gain=g)
        torch.cuda.synchronize()
        gains.append(g.cpu().numpy())
    assert np.array_equal(gains[0].view(np.uint32), gains[1].view(np.uint32))
    sel = np.array([3, 17, 0, 11], dtype=np.int32)
    g = torch.full((B, K), -7.0, dtype=torch.float32, device=dev)
    Yt = torch.from_numpy(wl3.Y.astype(np.complex64)).to(dev)
    fp.detect(Ht, Yt, st, 64, 11, 4, "fp16", variant=2, gain=g, chan_idx=torch.from_numpy(sel).to(dev))
    torch.cuda.synchronize()
    gi = g.cpu().numpy()
    assert np.array_equal(gi[sel].view(np.uint32), gains[0][sel].view(np.uint32))
    assert np.all(np.delete(gi, sel, axis=0) == -7.0)


def test_gain_fp8_large_k_with_refinement():
    """K = 128, fp8 operands, L = 16, one FP64 refinement step (the c4 schedule):
    gains against the oracle's from its own u_W Gram."""
    wl = W.draw(6, 512, 128, 14, 256, 25.0, 0.9, 0.9, seed=95)
    _say("case gain fp8 K=128 L=16 refine 1")
    _, g, _ = _gain_gpu_sched(wl, np.complex64, 256, 32, 16, "fp8", refine=1)
    r1 = oracle_detect(wl, 256, 32, 16, "fp8", io=np.complex64, refine=1, accum="exact")
    r2 = oracle_detect(wl, 256, 32, 16, "fp8", io=np.complex64, refine=1, accum="sequential")
    g1 = DM.effective_gain(r1.A, wl.sigma2, 16, "fp32")
    spread = np.abs(g1 - DM.effective_gain(r2.A, wl.sigma2, 16, "fp32")).max()
    tol = 4 * spread + 16 * 16 * 2.0**-24
    _say(f"  gain gpu-oracle max {np.abs(g - g1).max():.2e}, oracle order spread {spread:.2e}")
    assert np.all(np.abs(g - g1) <= tol)


def _gain_gpu_sched(wl, io, qam, iters, L, sched, refine=0, variant=0):
    import torch

    import paper_2504_09820_amd as fp

    dev = torch.device("cuda:0")
    Ht = torch.from_numpy(np.ascontiguousarray(wl.H.astype(io))).to(dev)
    Yt = torch.from_numpy(np.ascontiguousarray(wl.Y.astype(io))).to(dev)
    st = torch.from_numpy(np.ascontiguousarray(wl.sigma2)).to(dev)
    B, _, K = wl.H.shape
    gain = torch.full((B, K), -7.0, dtype=torch.float32, device=dev)
    x, lab, fl = fp.detect(Ht, Yt, st, qam, iters, L, sched, refine_steps=refine, variant=variant, gain=gain)
    torch.cuda.synchronize()
    return x.cpu().numpy().astype(np.complex128), gain.cpu().numpy().astype(np.float64), fl.cpu().numpy()


def test_binding_rejects_mismatched_outputs():
    """Caller-supplied outputs of the wrong shape, dtype or layout are
    rejected before any launch (the kernels write at the sizes the call implies)."""
    import torch

    import paper_2504_09820_amd as fp

    dev = torch.device("cuda:0")
    wl = W.draw(4, 32, 8, 3, 16, 15.0, 0.3, 0.3, seed=96)
    H = torch.from_numpy(wl.H.astype(np.complex64)).to(dev)
    Y = torch.from_numpy(wl.Y.astype(np.complex64)).to(dev)
    s2 = torch.from_numpy(wl.sigma2).to(dev)
    good = (torch.empty((4, 8, 3), dtype=torch.complex64, device=dev), torch.empty((4, 8, 3), dtype=torch.uint8, device=dev),
            torch.empty((4,), dtype=torch.int32, device=dev))
    bad = [(torch.empty((4, 8, 2), dtype=torch.complex64, device=dev),) + good[1:],
           (good[0].to(torch.complex128),) + good[1:],
           (good[0], good[1][:, :, :2], good[2]),
           (good[0], good[1], torch.empty((3,), dtype=torch.int32, device=dev)),
           (torch.empty((4, 3, 8), dtype=torch.complex64, device=dev).transpose(1, 2),) + good[1:]]
    for o in bad:
        with pytest.raises((TypeError, ValueError)):
            fp.detect(H, Y, s2, 16, 4, 4, "fp16", out=o)
    with pytest.raises((TypeError, ValueError)):
        fp.detect(H, Y, s2, 16, 4, 4, "fp16", gain=torch.empty((4, 7), dtype=torch.float32, device=dev))
    x, _, _ = fp.detect(H, Y, s2, 16, 4, 4, "fp16", out=good)
    g = torch.full((4, 8), 0.5, dtype=torch.float32, device=dev)
    for o in (torch.empty((4, 8, 3, 2), dtype=torch.float32, device=dev),
              torch.empty((4, 8, 3, 4), dtype=torch.float64, device=dev)):
        with pytest.raises((TypeError, ValueError)):
            fp.demap_maxlog(x, g, 16, out=o)
    with pytest.raises(TypeError):
        fp.demap_maxlog(x.real.contiguous(), g, 16)
    with pytest.raises(TypeError):
        fp.slice_qam(x.real.contiguous(), 16)
    torch.cuda.synchronize()


def _quant8(llr32, scale):
    """round(LLR * scale) to nearest even in FP32, NaN -> 0, clamped to +-127."""
    with np.errstate(invalid="ignore", over="ignore"):
        t = np.asarray(llr32, dtype=np.float32) * np.float32(scale)
    t = np.where(np.isnan(t), np.float32(0), t)
    return np.clip(np.rint(t), -127, 127).astype(np.int8)


@pytest.mark.parametrize("io", [np.complex64, np.complex128])
@pytest.mark.parametrize("q", [4, 16, 64, 256])
def test_demap_int8(q, io):
    """8-bit LLRs: bitwise the quantisation of the float demapper's own output
    (same FP32 product and rounding), and within one step of the quantised
    oracle LLRs; saturation, NaN -> 0 and the degenerate gains included."""
    import torch

    import paper_2504_09820_amd as fp

    rng = np.random.default_rng(40 + q + (io == np.complex128))
    B, K, R = 9, 7, 11                                    # 693 symbols, ragged
    x = ((rng.standard_normal((B, K, R)) + 1j * rng.standard_normal((B, K, R))) * 0.9).astype(io)
    gain = rng.uniform(0.02, 0.999, (B, K)).astype(np.float32)
    gain[0, :3] = [0.0, 1.0, 0.9999]                      # no signal, zero-forcing (+-inf), huge LLRs (saturate)
    gain[1, 0] = np.nan
    x[2, 0, 0] = np.nan
    _say(f"case demap int8 q={q} io={np.dtype(io).name}")
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(x).to(dev)
    gt = torch.from_numpy(gain).to(dev)
    for scale in (4.0, 0.37):
        l32 = fp.demap_maxlog(xt, gt, q)
        l8 = fp.demap_maxlog(xt, gt, q, scale=scale)
        torch.cuda.synchronize()
        got = l8.cpu().numpy()
        assert got.dtype == np.int8
        np.testing.assert_array_equal(got, _quant8(l32.cpu().numpy(), scale))
        ref = DM.maxlog_llr(x.astype(np.complex128), gain.astype(np.float64)[..., None], q)
        qo = _quant8(ref.astype(np.float32), scale).astype(np.int32)
        assert np.max(np.abs(got.astype(np.int32) - qo)) <= 1
        assert np.all(got[np.isnan(ref)] == 0)
    assert np.any(np.abs(got) == 127)                     # saturation was exercised
