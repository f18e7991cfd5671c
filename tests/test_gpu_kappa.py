"""Per-channel condition-number estimates (the kappa output of
fpcg_detect_ex) and launches over channel subsets, through the C ABI
binding: the GPU estimate against the oracle's Lanczos estimate from its own
CG coefficients (and against the spectrum where the Krylov space is full),
indexed launches bitwise equal to the full launch on their channels, and
per-channel format groups (precision.detect_adaptive)."""
import sys

import numpy as np
import pytest

import workload as W
from oracle import detect as D
from tests.gpu_common import oracle_sched

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _wl(B, Nbs, K, R, q, snr, zeta, seed):
    return W.draw(B, Nbs, K, R, q, snr, zeta, zeta, seed=seed)


def _run(wl, io, qam, iters, L, sched, variant=0, chan_idx=None, H=None, Y=None):
    import torch

    import paper_2504_09820_amd as fp

    dev = torch.device("cuda:0")
    Hn = wl.H if H is None else H
    Yn = wl.Y if Y is None else Y
    Ht = torch.from_numpy(np.ascontiguousarray(Hn.astype(io))).to(dev)
    Yt = torch.from_numpy(np.ascontiguousarray(Yn.astype(io))).to(dev)
    st = torch.from_numpy(np.ascontiguousarray(wl.sigma2)).to(dev)
    B, _, K = Hn.shape
    R = Yn.shape[2]
    # sentinels: what an indexed launch must leave untouched
    out = (torch.full((B, K, R), 7.0 + 7.0j, dtype=Ht.dtype, device=dev),
           torch.full((B, K, R), 255, dtype=torch.uint8, device=dev),
           torch.full((B,), -1, dtype=torch.int32, device=dev))
    kap = torch.full((B,), -1.0, dtype=torch.float32, device=dev)
    idx = None if chan_idx is None else torch.from_numpy(np.asarray(chan_idx, dtype=np.int32)).to(dev)
    fp.detect(Ht, Yt, st, qam, iters, L, sched, variant=variant, out=out, chan_idx=idx, kappa=kap)
    torch.cuda.synchronize()
    return (out[0].cpu().numpy(), out[1].cpu().numpy(), out[2].cpu().numpy(), kap.cpu().numpy().astype(np.float64))


def _oracle_kappa(wl, io, qam, iters, L, name, variant=0, accum="exact", H=None, Y=None):
    Hn = (wl.H if H is None else H).astype(io).astype(np.complex128)
    Yn = (wl.Y if Y is None else Y).astype(io).astype(np.complex128)
    co = []
    D.detect(Hn, Yn, wl.sigma2, qam, iters, L, oracle_sched(name, variant=variant, accum=accum), coeffs=co)
    # the device estimate uses the first four received vectors
    return D.lanczos_kappa(co, R_valid=min(Yn.shape[2], 4)) if co else np.full(Hn.shape[0], np.nan)


def _spectrum_kappa(wl, io, L):
    H = wl.H.astype(io).astype(np.complex128)
    K = H.shape[2]
    A = np.conj(np.swapaxes(H, -1, -2)) @ H + wl.sigma2[:, None, None] * np.eye(K)
    if L:
        T, _ = D.bj_factor(A, L)
        A = T @ A @ np.conj(np.swapaxes(T, -1, -2))
    ev = np.linalg.eigvalsh(A)
    return ev[:, -1] / ev[:, 0]


# multisection of the extreme Ritz values: the upper bracket shrunk 19683-fold and
# the lower one's logarithm 177147-fold, on coefficients recorded in fp32
RTOL = 2e-3


def test_kappa_fp64_full_krylov_space():
    wl = _wl(24, 128, 32, 14, 64, 20.0, 0.5, 3)
    _say("case kappa fp64 K=32 I=32")
    _, _, fl, kg = _run(wl, np.complex128, 64, 32, 0, "fp64")
    ko = _oracle_kappa(wl, np.complex128, 64, 32, 0, "fp64")
    ks = _spectrum_kappa(wl, np.complex128, 0)
    _say(f"  kappa gpu {np.round(kg[:4], 3)} oracle {np.round(ko[:4], 3)} spectrum {np.round(ks[:4], 3)}")
    assert np.all(fl == 0)
    np.testing.assert_allclose(kg, ko, rtol=RTOL)
    np.testing.assert_allclose(kg, ks, rtol=1e-2)                 # I = K: the Ritz values are the spectrum


@pytest.mark.parametrize("sched,L,variant,iters,R", [("fp16", 4, 2, 11, 14), ("bf16", 8, 0, 12, 37), ("fp32", 4, 1, 10, 5)])
def test_kappa_reduced_precision_matches_oracle(sched, L, variant, iters, R):
    wl = _wl(12, 96, 32, R, 64, 20.0, 0.5, 4)
    _say(f"case kappa {sched} L={L} v{variant} I={iters} R={R}")
    _, _, _, kg = _run(wl, np.complex64, 64, iters, L, sched, variant)
    ke = _oracle_kappa(wl, np.complex64, 64, iters, L, sched, variant, accum="exact")
    kq = _oracle_kappa(wl, np.complex64, 64, iters, L, sched, variant, accum="sequential")
    ks = _spectrum_kappa(wl, np.complex64, L)
    # the GPU is a third valid rounding order of the same coefficients
    dev = np.abs(kg - ke) / ke
    spread = np.abs(kq - ke) / ke
    _say(f"  rel. distance gpu-oracle max {dev.max():.2e}, oracle order spread max {spread.max():.2e}")
    assert np.all(dev <= 4 * spread + RTOL)
    assert np.all(kg <= ks * (1 + RTOL))                          # Ritz values inside the spectrum
    assert np.all(kg >= 1.0)


def test_kappa_without_steps_is_nan():
    wl = _wl(6, 64, 16, 3, 16, 15.0, 0.3, 5)
    _, _, _, k0 = _run(wl, np.complex128, 16, 0, 4, "fp64")
    assert np.all(np.isnan(k0))
    # a channel whose received vectors are zero: rho = 0 freezes every column before its first step
    Y = wl.Y.copy()
    Y[2] = 0
    _, _, fl, kz = _run(wl, np.complex128, 16, 8, 4, "fp64", Y=Y)
    assert np.isnan(kz[2]) and np.all(np.isfinite(np.delete(kz, 2)))
    assert fl[2] & D.FLAG_BREAKDOWN


@pytest.mark.parametrize("sched,L,variant,R", [("fp16", 4, 2, 14), ("fp64", 0, 0, 14), ("bf16", 8, 0, 21)])
def test_indexed_launch_matches_full_launch(sched, L, variant, R):
    B = 40
    wl = _wl(B, 128, 32, R, 64, 18.0, 0.5, 6)
    io = np.complex128 if sched == "fp64" else np.complex64
    rng = np.random.default_rng(1)
    sel = rng.permutation(B)[:17]
    idx = np.concatenate([sel[:8], [-1, B + 5], sel[8:]])        # two indices outside the batch are skipped
    _say(f"case indexed launch {sched} L={L} R={R}: {len(sel)} of {B} channels")
    xf, lf, ff, kf = _run(wl, io, 64, 12, L, sched, variant)
    xi, li, fi, ki = _run(wl, io, 64, 12, L, sched, variant, chan_idx=idx)
    rest = np.setdiff1d(np.arange(B), sel)
    assert np.array_equal(xi[sel].view(np.uint8), xf[sel].view(np.uint8))
    assert np.array_equal(li[sel], lf[sel]) and np.array_equal(fi[sel], ff[sel])
    assert np.array_equal(ki[sel], kf[sel])
    assert np.all(xi[rest] == 7.0 + 7.0j) and np.all(li[rest] == 255) and np.all(fi[rest] == -1)
    assert np.all(ki[rest] == -1.0)


def test_adaptive_formats_run_each_group_in_its_format():
    import torch

    import paper_2504_09820_amd as fp
    from paper_2504_09820_amd import precision

    B, Nbs, K, R = 48, 256, 64, 14
    wl = W.draw(B, Nbs, K, R, 64, 15.0, 0.0, 0.0, seed=8)
    # mixed conditioning: half the channels strongly correlated
    wl2 = W.draw(B, Nbs, K, R, 64, 15.0, 0.9, 0.9, seed=9)
    H = np.where((np.arange(B) % 2 == 0)[:, None, None], wl.H, wl2.H)
    Y = np.where((np.arange(B) % 2 == 0)[:, None, None], wl.Y, wl2.Y)
    dev = torch.device("cuda:0")
    Ht = torch.from_numpy(H.astype(np.complex64)).to(dev)
    Yt = torch.from_numpy(Y.astype(np.complex64)).to(dev)
    st = torch.from_numpy(wl.sigma2).to(dev)
    kap = torch.empty((B,), dtype=torch.float32, device=dev)
    fp.detect(Ht, Yt, st, 64, 16, 8, "fp32", variant=2, kappa=kap)
    fmts = precision.formats_per_channel(kap, K, allowed=("fp16", "fp32"))
    _say(f"case adaptive formats: {dict(zip(*np.unique(fmts.astype(str), return_counts=True)))}")
    assert len(set(fmts)) == 2                                    # both groups present
    x, lab, fl, groups = precision.detect_adaptive(Ht, Yt, st, 64, 16, 8, fmts, variant=2)
    torch.cuda.synchronize()
    for name, n in groups.items():
        sel = np.nonzero(fmts == name)[0]
        xr, lr, fr = fp.detect(Ht, Yt, st, 64, 16, 8, name, variant=2)
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy()[sel].view(np.uint8), xr.cpu().numpy()[sel].view(np.uint8)), name
        assert np.array_equal(lab.cpu().numpy()[sel], lr.cpu().numpy()[sel]), name
        assert n == sel.size
