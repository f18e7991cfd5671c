"""Robustness workload generators (Sec. V: imperfect CSI, geometry-based and
Gauss-Markov time-varying channels): their defining statistics."""
import math

import numpy as np
import pytest
from scipy.special import j0

import workload as W


def test_imperfect_csi_error_power_and_true_channel():
    wl = W.draw(400, 64, 8, 3, 16, 20.0, 0.5, 0.5, seed=1)
    for eps in (20.0, 25.0):
        w = W.imperfect_csi(wl, eps, seed=2)
        ratio = np.mean(np.abs(w.H - w.H_true) ** 2) / np.mean(np.abs(w.H_true) ** 2)
        assert ratio == pytest.approx(10 ** (-eps / 10), rel=0.02)
        assert np.array_equal(w.H_true, wl.H) and np.array_equal(w.Y, wl.Y)   # Y keeps the true channel


def test_gauss_markov_correlation_is_bessel():
    fd, tau = 1000.0, 1.0 / 14000.0
    rho = j0(2 * math.pi * fd * tau)
    assert rho == pytest.approx(0.95028, abs=1e-5)
    steps = W.gauss_markov(4000, 16, 4, 2, 16, 20.0, 0.5, 0.5, 4, fd, tau, seed=3)
    p0 = np.mean(np.abs(steps[0].H) ** 2)
    for a, b in zip(steps, steps[1:]):
        c = np.real(np.mean(b.H * np.conj(a.H))) / p0
        assert c == pytest.approx(rho, abs=0.01)
        assert np.mean(np.abs(b.H) ** 2) == pytest.approx(p0, rel=0.02)       # stationary power
    # each step's Y is drawn with that step's channel and symbols
    r = steps[2].Y - steps[2].H @ steps[2].X
    assert np.mean(np.abs(r) ** 2) == pytest.approx(steps[2].sigma2[0], rel=0.05)


def test_geometry_paths_and_power():
    g = W.geometry(3000, 32, 4, 1, 16, 20.0, paths=5, mu=1.0, seed=4)
    assert np.mean(np.sum(np.abs(g.H) ** 2, axis=1)) == pytest.approx(1.0, rel=0.03)
    # one path: every column is a scaled array response, consecutive entries
    # share one modulus and one phase step
    g1 = W.geometry(50, 16, 3, 1, 16, 20.0, paths=1, seed=5)
    ratio = g1.H[:, 1:, :] / g1.H[:, :-1, :]
    np.testing.assert_allclose(np.abs(ratio), 1.0, rtol=1e-12)
    np.testing.assert_allclose(ratio, ratio[:, :1, :] * np.ones_like(ratio), rtol=1e-10)
