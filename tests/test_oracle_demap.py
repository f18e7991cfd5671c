"""Pins of the soft-output oracle (oracle.demap) against closed forms, the exact
LMMSE gain, simulation and the max-log error bound."""
import math

import numpy as np
import pytest

from oracle import demap as DM
from oracle import detect as D

QS = (4, 16, 64, 256)


@pytest.mark.parametrize("q", QS)
def test_constellation_energy_labels_gray(q):
    pts, lab = DM.constellation(q)
    assert pts.size == q and np.mean(np.abs(pts) ** 2) == pytest.approx(1.0, rel=1e-14)
    assert np.array_equal(np.sort(lab), np.arange(q))
    # nearest neighbours (one level step on one axis) differ in exactly one label bit
    m = int(math.isqrt(q))
    step = 2.0 / math.sqrt(2.0 * (q - 1) / 3.0)
    d = np.abs(pts[:, None] - pts[None, :])
    nb = np.isclose(d, step, rtol=1e-12)
    assert nb.sum() == 2 * 2 * m * (m - 1)
    flips = np.bitwise_xor(lab[:, None], lab[None, :])[nb]
    assert np.all((flips & (flips - 1)) == 0) and np.all(flips > 0)
    # the slicer maps each point to its own label
    assert np.array_equal(D.slice_qam(pts, q), lab)


def test_qpsk_closed_form():
    # levels -1/sqrt2 (bit 0) and +1/sqrt2 (bit 1) per axis:
    # LLR = ((v - mu a1)^2 - (v - mu a0)^2) / (mu (1 - mu)) = -2 sqrt2 v / (1 - mu)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(500) + 1j * rng.standard_normal(500)
    mu = rng.uniform(0.05, 0.95, 500)
    llr = DM.maxlog_llr(x, mu, 4)
    np.testing.assert_allclose(llr[:, 0], -2 * math.sqrt(2) * x.real / (1 - mu), rtol=1e-12)
    np.testing.assert_allclose(llr[:, 1], -2 * math.sqrt(2) * x.imag / (1 - mu), rtol=1e-12)
    # for QPSK the max-log LLR is exact (one point per bit value and axis)
    np.testing.assert_allclose(DM.logmap_llr(x, mu, 4), llr, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("q", QS)
def test_signs_are_the_hard_decision(q):
    rng = np.random.default_rng(q)
    x = (rng.standard_normal(4000) + 1j * rng.standard_normal(4000)) * 0.8
    mu = rng.uniform(0.1, 0.99, 4000)
    llr = DM.maxlog_llr(x, mu, q)
    nb = llr.shape[-1]
    bits = (llr < 0).astype(np.int64)
    lab = np.zeros(4000, dtype=np.int64)
    for t in range(nb):
        lab |= bits[:, t] << (nb - 1 - t)
    np.testing.assert_array_equal(lab, D.slice_qam(x / mu, q))


@pytest.mark.parametrize("q", QS)
def test_maxlog_within_log_bound_of_exact(q):
    # log sum_i exp(-d_i) lies in [-min d, -min d + ln n]: the max-log LLR is
    # within ln(Q/2) of the exact one, and the gap vanishes at high SNR
    rng = np.random.default_rng(10 + q)
    pts, _ = DM.constellation(q)
    s = pts[rng.integers(0, q, 3000)]
    for mu, bound in ((0.6, math.log(q / 2)), (0.999, None)):
        nu = math.sqrt(mu * (1 - mu))
        x = mu * s + nu * (rng.standard_normal(3000) + 1j * rng.standard_normal(3000)) / math.sqrt(2)
        a, b = DM.maxlog_llr(x, mu, q), DM.logmap_llr(x, mu, q)
        if bound is not None:
            assert np.max(np.abs(a - b)) <= bound + 1e-9
        else:
            assert np.median(np.abs(a - b) / np.abs(b)) < 1e-3


def test_exact_llrs_are_calibrated():
    # simulate the model: the fraction of bits whose LLR sign is wrong must be
    # 1 / (1 + e^|L|) inside bins of |L| (the exact posterior's definition)
    q, n, mu = 16, 200000, 0.8
    rng = np.random.default_rng(3)
    pts, lab = DM.constellation(q)
    idx = rng.integers(0, q, n)
    nu = math.sqrt(mu * (1 - mu))
    x = mu * pts[idx] + nu * (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2)
    L = DM.logmap_llr(x, mu, q)
    bits = np.stack([(lab[idx] >> (3 - t)) & 1 for t in range(4)], axis=-1)
    wrong = (L > 0) == (bits == 1)
    a = np.abs(L).ravel()
    w = wrong.ravel()
    for lo, hi in ((0.0, 0.5), (0.5, 1.5), (1.5, 3.0)):
        sel = (a >= lo) & (a < hi)
        pred = np.mean(1.0 / (1.0 + np.exp(a[sel])))
        sd = math.sqrt(pred * (1 - pred) / sel.sum())
        assert abs(np.mean(w[sel]) - pred) < 5 * sd + 1e-3, (lo, hi)


def _gram(H, s2):
    Hh = np.conj(np.swapaxes(H, -1, -2))
    return Hh @ H + s2[:, None, None] * np.eye(H.shape[-1]), Hh @ H


def test_gain_exact_lmmse_and_no_preconditioner():
    rng = np.random.default_rng(4)
    H = (rng.standard_normal((6, 16, 8)) + 1j * rng.standard_normal((6, 16, 8))) / math.sqrt(32)
    s2 = rng.uniform(0.05, 0.5, 6)
    A, G = _gram(H, s2)
    # one block: M = A^{-1}, mu_k = (A^{-1} H^H H)_kk
    ref = np.real(np.diagonal(np.linalg.inv(A) @ G, axis1=1, axis2=2))
    np.testing.assert_allclose(DM.effective_gain(A, s2, 8), ref, rtol=1e-12)
    # no preconditioner: mu_k = G_kk / A_kk
    np.testing.assert_allclose(DM.effective_gain(A, s2, 0),
                               np.real(np.diagonal(G, axis1=1, axis2=2) / np.diagonal(A, axis1=1, axis2=2)),
                               rtol=1e-12)
    # 2 x 2 blocks: (A_i^{-1})_00 = a_11 / det(A_i)
    mu2 = DM.effective_gain(A, s2, 2)
    for c in range(6):
        for b0 in range(0, 8, 2):
            a00, a11, a01 = A[c, b0, b0].real, A[c, b0 + 1, b0 + 1].real, A[c, b0, b0 + 1]
            det = a00 * a11 - abs(a01) ** 2
            assert mu2[c, b0] == pytest.approx(1 - s2[c] * a11 / det, rel=1e-12)
            assert mu2[c, b0 + 1] == pytest.approx(1 - s2[c] * a00 / det, rel=1e-12)


def test_gain_and_error_variance_by_simulation():
    # x_hat = A^{-1} H^H y with unit-energy symbols and noise of variance
    # sigma^2: E[x_hat_k s_k^*] = mu_k and E|x_hat_k - mu_k s_k|^2 = mu_k (1 - mu_k)
    rng = np.random.default_rng(5)
    K, M, n, s2 = 4, 8, 100000, 0.3
    H = (rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))) / math.sqrt(2 * M)
    pts, _ = DM.constellation(16)
    S = pts[rng.integers(0, 16, (K, n))]
    Y = H @ S + math.sqrt(s2 / 2) * (rng.standard_normal((M, n)) + 1j * rng.standard_normal((M, n)))
    A, _ = _gram(H[None], np.array([s2]))
    X = np.linalg.solve(A[0], np.conj(H.T) @ Y)
    mu = DM.effective_gain(A, np.array([s2]), K)[0]
    np.testing.assert_allclose(np.real(np.mean(X * np.conj(S), axis=1)), mu, atol=0.01)
    np.testing.assert_allclose(np.mean(np.abs(X - mu[:, None] * S) ** 2, axis=1), mu * (1 - mu), rtol=0.03)


def test_degenerate_gains():
    x = np.array([0.3 + 0.1j, -0.2 + 0.7j, 0.0 + 0.0j])
    z = DM.maxlog_llr(x, np.zeros(3), 16)
    assert np.all(z == 0)                                     # nothing received: no information
    one = DM.maxlog_llr(x[:2], np.ones(2), 16)
    assert np.all(np.isinf(one))                              # zero-forcing: certainty
    lab = D.slice_qam(x[:2], 16)
    for t in range(4):
        np.testing.assert_array_equal(one[:, t] < 0, ((lab >> (3 - t)) & 1) == 1)
    assert np.all(np.isnan(DM.maxlog_llr(x, np.array([np.nan, 0.5, 0.5]), 16)[0]))
    assert np.all(np.isnan(DM.maxlog_llr(np.array([np.nan + 0j]), np.array([0.5]), 16)))
    # gains outside [0, 1] (rounding) are clamped
    np.testing.assert_array_equal(DM.maxlog_llr(x, np.array([-1e-9, 1.0 + 1e-9, 0.0]), 16)[[0, 2]],
                                  DM.maxlog_llr(x, np.array([0.0, 1.0, 0.0]), 16)[[0, 2]])
