"""fpcg_detect_ex_static (no allocation; the kappa record in a static per-GPU
array) against fpcg_detect_ex on the same inputs: bitwise identical x_hat,
labels, flags, kappa estimates and gains, on two calls in a row (the second
smaller, and with a channel subset), and the size limit refused on the host."""
import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu


def _run(fp, ctx, wl, static, L, sched, iters, idx=None):
    import torch

    dev = torch.device("cuda:0")
    H = torch.from_numpy(wl.H.astype(np.complex64)).to(dev)
    Y = torch.from_numpy(wl.Y.astype(np.complex64)).to(dev)
    s2 = torch.from_numpy(wl.sigma2).to(dev)
    B, _, K = H.shape
    kap = torch.full((B,), -1.0, dtype=torch.float32, device=dev)
    gain = torch.full((B, K), -1.0, dtype=torch.float32, device=dev)
    out = (torch.zeros((B, K, Y.shape[2]), dtype=torch.complex64, device=dev),
           torch.zeros((B, K, Y.shape[2]), dtype=torch.uint8, device=dev), torch.zeros((B,), dtype=torch.int32, device=dev))
    ci = None if idx is None else torch.from_numpy(np.asarray(idx, dtype=np.int32)).to(dev)
    fp.detect(H, Y, s2, 64, iters, L, sched, variant=2 if L else 0, ctx=ctx, out=out, chan_idx=ci, kappa=kap,
              gain=gain, static_workspace=static)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (*out, kap, gain)]


def test_static_workspace_matches_allocating_entry_point():
    import paper_2504_09820_amd as fp

    ctx = fp.Context(0)
    big = W.draw(900, 128, 32, 14, 64, 20.0, 0.5, 0.5, seed=71)
    small = W.draw(150, 256, 64, 20, 64, 15.0, 0.7, 0.7, seed=72)
    for wl, L, sched, iters, idx in ((big, 4, "fp16", 11, None), (small, 8, "fp32", 16, [3, 0, 149, 77, 200, -1])):
        print(f"case no-alloc B={wl.H.shape[0]} K={wl.H.shape[2]} L={L} {sched} idx={idx is not None}", flush=True)
        a = _run(fp, ctx, wl, True, L, sched, iters, idx)
        b = _run(fp, ctx, wl, False, L, sched, iters, idx)
        for u, v in zip(a, b):
            assert np.array_equal(u.view(np.uint8), v.view(np.uint8))
        assert np.all(np.isfinite(a[3][0 if idx is None else 3]))
    ctx.close()


def test_static_workspace_limit_is_refused():
    import torch

    import paper_2504_09820_amd as fp

    ctx = fp.Context(0)
    dev = torch.device("cuda:0")
    B, Nbs, K, R, it = 70000, 16, 8, 4, 8       # 70000 * 4 * 8 * 8 bytes > 16 MiB
    H = torch.zeros((B, Nbs, K), dtype=torch.complex64, device=dev)
    Y = torch.zeros((B, Nbs, R), dtype=torch.complex64, device=dev)
    s2 = torch.ones((B,), dtype=torch.float64, device=dev)
    kap = torch.empty((B,), dtype=torch.float32, device=dev)
    with pytest.raises(fp.FpcgError) as e:
        fp.detect(H, Y, s2, 16, it, 0, "fp32", ctx=ctx, kappa=kap, static_workspace=True)
    assert e.value.status == -1 and "static workspace" in str(e.value)
    ctx.close()
