"""Continuous-batching request loop (fpcg_server_*): requests of mixed shapes
and schedules submitted together run overlapped on the device, and every
request's result is bitwise the one the same request gives alone (each
channel is computed by its own workgroup in a fixed order)."""
from __future__ import annotations

import sys
import time

import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


SHAPES = [(64, 8), (64, 16), (64, 32), (128, 8), (128, 16), (128, 32), (128, 64), (256, 16), (256, 32), (256, 64)]
SCHEDS = [("fp16", 4, 2, 0), ("fp32", 0, 0, 0), ("bf16", 8, 2, 0), ("fp64", 0, 0, 0), ("fp16", 8, 0, 4), ("fp8", 4, 2, 0)]


def _requests(n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        Nbs, K = SHAPES[rng.integers(len(SHAPES))]
        sched, L, v, refresh = SCHEDS[rng.integers(len(SCHEDS))]
        if L and K % L:
            L = 4
        if sched == "fp8" and K < 32:
            sched = "fp16"
        B = int(rng.integers(1, 120))
        q = int(rng.choice([16, 64]))
        wl = W.draw(B, Nbs, K, 14, q, float(rng.uniform(5, 25)), float(rng.uniform(0, 0.9)),
                    float(rng.uniform(0, 0.9)), seed=1000 + i)
        io = np.complex128 if sched == "fp64" else np.complex64
        reqs.append(dict(H=wl.H.astype(io), Y=wl.Y.astype(io), s2=wl.sigma2, q=q, iters=int(rng.integers(4, 17)), L=L,
                         sched=sched, variant=v, refresh=refresh))
    return reqs


def _alone(fp, r):
    import torch

    dev = torch.device("cuda:0")
    x, lab, fl = fp.detect(torch.from_numpy(r["H"]).to(dev), torch.from_numpy(r["Y"]).to(dev),
                           torch.from_numpy(r["s2"]).to(dev), r["q"], r["iters"], r["L"], r["sched"],
                           refresh_every=r["refresh"], variant=r["variant"])
    torch.cuda.synchronize()
    return x.cpu().numpy(), lab.cpu().numpy(), fl.cpu().numpy().astype(np.uint32)


def _serve(fp, reqs, budget, n_slots):
    ctx = fp.Context(0, budget)
    srv = fp.Server(ctx, n_slots=n_slots, queue_cap=len(reqs))
    tickets = [srv.submit(r["H"], r["Y"], r["s2"], r["q"], r["iters"], r["L"], r["sched"],
                          refresh_every=r["refresh"], variant=r["variant"]) for r in reqs]
    out = {}
    max_flight, max_held = 0, 0
    t0 = time.time()
    while len(out) < len(tickets):
        fl_, q_, held = srv.stats()
        max_flight, max_held = max(max_flight, fl_), max(max_held, held)
        for t in tickets:
            if t not in out:
                res = srv.poll(t)
                if res is not None:
                    out[t] = res
        assert time.time() - t0 < 60, "serving did not finish"
    srv.close()
    ctx.close()
    return [out[t] for t in tickets], max_flight, max_held


def _check_same(reqs, alone, served):
    for i, (r, a, s) in enumerate(zip(reqs, alone, served)):
        assert np.array_equal(a[0].view(np.uint8), s[0].view(np.uint8)), f"request {i} x_hat differs"
        assert np.array_equal(a[1], s[1]), f"request {i} labels differ"
        assert np.array_equal(a[2], s[2]), f"request {i} flags differ"


def test_mixed_requests_match_alone_bitwise():
    import paper_2504_09820_amd as fp

    reqs = _requests(14, 7)
    _say("case serving: 14 mixed requests, 4 slots, default budget")
    alone = [_alone(fp, r) for r in reqs]
    served, max_flight, _ = _serve(fp, reqs, 0, 4)
    _say(f"  max in flight {max_flight}")
    _check_same(reqs, alone, served)
    assert max_flight >= 2          # requests overlapped on the device


def test_small_budget_admits_as_memory_frees():
    import paper_2504_09820_amd as fp

    reqs = _requests(10, 11)
    sizes = []
    for r in reqs:
        B, Nbs, K = r["H"].shape
        el = r["H"].itemsize
        sizes.append(B * (Nbs * K + Nbs * 14 + K * 14) * el + B * (8 + K * 14 + 4) + 6 * 256)
    budget = int(2.2 * max(sizes))
    _say(f"case serving: 10 requests, budget {budget} bytes (about two of the largest)")
    alone = [_alone(fp, r) for r in reqs]
    served, max_flight, max_held = _serve(fp, reqs, budget, 8)
    _say(f"  max in flight {max_flight}, max device bytes held {max_held}")
    _check_same(reqs, alone, served)
    assert max_held <= budget


def test_resident_channel_sets_match_alone_bitwise():
    """Channel sets uploaded once; requests carry only Y (several blocks of
    received vectors per channel set) and match the direct launch bitwise;
    idle sets are released."""
    import paper_2504_09820_amd as fp

    reqs = _requests(6, 13)
    _say("case serving: 6 resident channel sets, 3 Y blocks each")
    ctx = fp.Context(0)
    srv = fp.Server(ctx, n_slots=4, queue_cap=64)
    handles = [srv.channels(r["H"], r["s2"]) for r in reqs]
    rng = np.random.default_rng(3)
    jobs = []
    for r, h in zip(reqs, handles):
        for blk in range(3):
            Yb = (r["Y"] * (1.0 + 0.25 * blk) + 0.01 * blk).astype(r["Y"].dtype)   # further received vectors
            jobs.append((r, h, Yb))
    order = rng.permutation(len(jobs))
    tickets = {}
    for i in order:
        r, h, Yb = jobs[i]
        tickets[i] = srv.submit(None, Yb, None, r["q"], r["iters"], r["L"], r["sched"], refresh_every=r["refresh"],
                                variant=r["variant"], channels=h)
    with pytest.raises(fp.FpcgError):
        srv.release(987654)                       # not a channel set
    out = {}
    t0 = time.time()
    while len(out) < len(jobs):
        for i, t in tickets.items():
            if i not in out:
                res = srv.poll(t)
                if res is not None:
                    out[i] = res
        assert time.time() - t0 < 60
    for i, (r, h, Yb) in enumerate(jobs):
        a = _alone(fp, dict(r, Y=Yb))
        s = out[i]
        assert np.array_equal(a[0].view(np.uint8), s[0].view(np.uint8)), f"job {i} x_hat differs"
        assert np.array_equal(a[1], s[1]) and np.array_equal(a[2], s[2]), f"job {i} labels/flags differ"
    _, _, held_before = srv.stats()
    for h in handles:
        srv.release(h)
    _, _, held = srv.stats()
    assert held < held_before
    srv.close()
    ctx.close()


def test_kept_factor_across_channel_updates():
    """A resident set keeps its block-Jacobi factor: the first request stores
    it, the rest (several in flight at once on other slots) read it and match
    the direct launch bitwise.  After fpcg_server_channels_update with the
    next Gauss-Markov realisation and keep_precond, requests match a direct
    launch of the new channels with the previous realisation's factor
    (fpcg_detect_pc load); after an update without it, a plain launch."""
    import torch

    import paper_2504_09820_amd as fp

    dev = torch.device("cuda:0")
    steps = W.gauss_markov(96, 128, 32, 14, 64, 20.0, 0.6, 0.6, steps=3, fd_hz=1000.0, seed=77)
    io = np.complex64
    q, it, L, sched, v = 64, 11, 4, "fp16", 2
    ctx = fp.Context(0)
    srv = fp.Server(ctx, n_slots=4, queue_cap=64)
    h = srv.channels(steps[0].H.astype(io), steps[0].sigma2)

    def serve(Ys):
        tickets = [srv.submit(None, Yb, None, q, it, L, sched, variant=v, channels=h) for Yb in Ys]
        out, t0 = {}, time.time()
        while len(out) < len(tickets):
            for t in tickets:
                if t not in out:
                    r = srv.poll(t)
                    if r is not None:
                        out[t] = r
            assert time.time() - t0 < 60
        return [out[t] for t in tickets]

    def direct(H, Y, s2, precond=None, mode=None):
        x, lab, fl = fp.detect(torch.from_numpy(H).to(dev), torch.from_numpy(Y).to(dev), torch.from_numpy(s2).to(dev),
                               q, it, L, sched, variant=v, precond=precond, precond_mode=mode)
        torch.cuda.synchronize()
        return x.cpu().numpy(), lab.cpu().numpy(), fl.cpu().numpy().astype(np.uint32)

    def same(a, s):
        assert np.array_equal(a[0].view(np.uint8), s[0].view(np.uint8))
        assert np.array_equal(a[1], s[1]) and np.array_equal(a[2], s[2])

    _say("case serving: kept factor, 5 blocks of received vectors per realisation, 3 realisations")
    H0, s0 = steps[0].H.astype(io), steps[0].sigma2
    Ys = [(steps[0].Y * (1.0 + 0.1 * k)).astype(io) for k in range(5)]
    for Yb, s in zip(Ys, serve(Ys)):
        same(direct(H0, Yb, s0), s)
    # the previous realisation's factor, as a direct launch would keep it
    T0 = torch.zeros((96, 32, L), dtype=torch.complex64, device=dev)
    direct(H0, Ys[0], s0, T0, "store")
    H1, s1 = steps[1].H.astype(io), steps[1].sigma2
    srv.channels_update(h, H1, s1, keep_precond=True)
    Ys = [(steps[1].Y * (1.0 + 0.1 * k)).astype(io) for k in range(5)]
    for Yb, s in zip(Ys, serve(Ys)):
        same(direct(H1, Yb, s1, T0, "load"), s)
    H2, s2 = steps[2].H.astype(io), steps[2].sigma2
    srv.channels_update(h, H2, s2, keep_precond=False)
    Ys = [steps[2].Y.astype(io)]
    same(direct(H2, Ys[0], s2), serve(Ys)[0])
    with pytest.raises(ValueError):
        srv.channels_update(h, H2[:5], s2[:5])
    srv.release(h)
    srv.close()
    ctx.close()
