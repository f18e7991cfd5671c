"""The seeded input generator: determinism, structure and normalisation."""
import math

import numpy as np
import pytest

import workload as W


def test_exp_corr_structure():
    r = W.exp_corr(5, 0.6)
    assert np.allclose(np.diag(r), 1)
    assert r[0, 3] == pytest.approx(0.6**3)
    assert np.array_equal(r, r.conj().T)
    assert np.array_equal(W.exp_corr(4, 0.0), np.eye(4))


def test_psd_sqrt_squares_back():
    r = W.exp_corr(16, 0.9)
    s = W.psd_sqrt(r)
    assert np.allclose(s @ s, r, atol=1e-12)
    assert np.allclose(s, s.conj().T, atol=1e-14)


@pytest.mark.parametrize("q", [4, 16, 64, 256])
def test_qam_unit_energy_and_grid(q):
    pts = W.qam_points(np.arange(q), q)
    assert np.mean(np.abs(pts) ** 2) == pytest.approx(1.0)
    assert len(set(np.round(pts, 12))) == q


def test_draw_is_deterministic_and_shaped():
    a = W.draw(5, 16, 4, 3, 16, 10.0, 0.5, 0.3, seed=4)
    b = W.draw(5, 16, 4, 3, 16, 10.0, 0.5, 0.3, seed=4)
    c = W.draw(5, 16, 4, 3, 16, 10.0, 0.5, 0.3, seed=5)
    assert a.H.shape == (5, 16, 4) and a.Y.shape == (5, 16, 3) and a.labels.shape == (5, 4, 3)
    assert np.array_equal(a.H, b.H) and np.array_equal(a.Y, b.Y) and np.array_equal(a.labels, b.labels)
    assert not np.array_equal(a.H, c.H)
    assert a.labels.min() >= 0 and a.labels.max() < 16


def test_channel_normalisation_and_snr():
    wl = W.draw(4000, 32, 4, 1, 4, 10.0, 0.0, 0.0, seed=1)
    assert np.mean(np.sum(np.abs(wl.H) ** 2, axis=1)) == pytest.approx(1.0, rel=0.02)   # E||h_k||^2 = 1
    assert wl.sigma2[0] == pytest.approx(0.1)
    wl2 = W.draw(10, 32, 4, 1, 4, 10.0, normalization="unit", seed=1)
    assert wl2.sigma2[0] == pytest.approx(3.2)
    n = wl.Y - wl.H @ wl.X
    assert np.mean(np.abs(n) ** 2) == pytest.approx(0.1, rel=0.05)
