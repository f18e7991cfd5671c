"""Zero-forcing (sigma^2 = 0 in eq. inversion) in the oracle: the direct solve
is the least-squares solution of H x = y (numpy lstsq), noise-free symbols
are recovered exactly, and CG / FP-BJ-CG reach the same solution when the
Krylov space is full."""
from __future__ import annotations

import numpy as np
import pytest

import workload as W
from oracle import detect as D


def _noise_free(B, Nbs, K, R, q, zeta, seed):
    wl = W.draw(B, Nbs, K, R, q, 30.0, zeta, zeta, seed=seed)
    Y = wl.H @ wl.X                                   # no noise
    return wl, Y


def test_zero_forcing_is_least_squares():
    rng = np.random.default_rng(0)
    H = rng.standard_normal((5, 20, 6)) + 1j * rng.standard_normal((5, 20, 6))
    Y = rng.standard_normal((5, 20, 3)) + 1j * rng.standard_normal((5, 20, 3))
    A, b = D.gram(H, Y, np.zeros(5))
    x = D.lmmse(A, b)
    ls = np.stack([np.linalg.lstsq(H[i], Y[i], rcond=None)[0] for i in range(5)])
    np.testing.assert_allclose(x, ls, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("L,variant", [(0, 0), (4, 0), (4, 1), (4, 2)])
def test_noise_free_symbols_recovered(L, variant):
    wl, Y = _noise_free(6, 48, 8, 4, 16, 0.5, 3)
    sched = D.schedule("fp64", variant=variant)
    res = D.detect(wl.H, Y, np.zeros(6), 16, 16, L, sched)   # I = 2K: converged
    np.testing.assert_allclose(res.xhat, wl.X, atol=1e-9)
    assert np.array_equal(res.labels, wl.labels)
    assert np.all(res.flags == 0)


def test_rank_deficient_zero_forcing_is_flagged():
    # K > Nbs: H^H H is singular; its block factorisation or the iteration breaks down
    rng = np.random.default_rng(1)
    H = rng.standard_normal((3, 4, 8)) + 1j * rng.standard_normal((3, 4, 8))
    Y = rng.standard_normal((3, 4, 2)) + 1j * rng.standard_normal((3, 4, 2))
    res = D.detect(H, Y, np.zeros(3), 16, 8, 8, D.schedule("fp64", variant=0))
    assert np.all(res.flags & (D.FLAG_BLOCK_NOT_PD | D.FLAG_BREAKDOWN))
