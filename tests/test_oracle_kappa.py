"""Pins of the oracle's per-channel condition-number estimate from the CG
coefficients (the Lanczos tridiagonal of CG): closed forms, exact-arithmetic
equalities with the spectrum of the iteration matrix, and Ritz-value
interlacing."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import detect as D


def _hpd(rng, B, K, cond):
    """B Hermitian positive definite K x K matrices with condition number cond."""
    Q, _ = np.linalg.qr(rng.standard_normal((B, K, K)) + 1j * rng.standard_normal((B, K, K)))
    ev = np.geomspace(1.0, cond, K)
    return (Q * ev[None, None, :]) @ np.conj(np.swapaxes(Q, -1, -2))


def _kappa(A):
    ev = np.linalg.eigvalsh(A)
    return ev[..., -1] / ev[..., 0]


def test_two_by_two_closed_form():
    # A = diag(1, 4), b = (1, 1): two exact CG steps, alpha_1 = 2/5,
    # beta_1 = 9/25, alpha_2 = 5/8; the tridiagonal has eigenvalues 1 and 4
    A = np.diag([1.0, 4.0]).astype(np.complex128)[None]
    b = np.ones((1, 2, 1), dtype=np.complex128)
    co = []
    D.fp_cg(A, b, 2, coeffs=co)
    np.testing.assert_allclose([co[0][0].item(), co[0][1].item(), co[1][0].item()], [0.4, 0.36, 0.625], rtol=1e-14)
    T = D.lanczos_tridiagonal([0.4, 0.625], [0.36, 0.0])
    np.testing.assert_allclose(np.linalg.eigvalsh(T), [1.0, 4.0], rtol=1e-13)
    assert D.lanczos_kappa(co)[0] == pytest.approx(4.0, rel=1e-13)


def test_full_krylov_space_gives_the_spectrum():
    rng = np.random.default_rng(1)
    A = _hpd(rng, 6, 8, 40.0)
    b = rng.standard_normal((6, 8, 3)) + 1j * rng.standard_normal((6, 8, 3))
    co = []
    D.fp_cg(A, b, 8, coeffs=co)
    np.testing.assert_allclose(D.lanczos_kappa(co), _kappa(A), rtol=1e-8)


def test_ritz_values_interlace():
    rng = np.random.default_rng(2)
    A = _hpd(rng, 5, 24, 300.0)
    b = rng.standard_normal((5, 24, 2)) + 1j * rng.standard_normal((5, 24, 2))
    co = []
    D.fp_cg(A, b, 12, coeffs=co)
    kap = _kappa(A)
    prev = np.zeros(5)
    for m in range(1, 13):
        k = D.lanczos_kappa(co[:m])
        assert np.all(k <= kap * (1 + 1e-10))         # inside the spectrum
        assert np.all(k >= prev * (1 - 1e-10))        # extremes move outward with m
        prev = k
    assert np.all(prev > 0.5 * kap)                   # the extremes converge first


def test_identity_scaled_matrix_takes_one_step():
    A = (3.0 * np.eye(5, dtype=np.complex128))[None]
    b = np.arange(1, 6, dtype=np.complex128).reshape(1, 5, 1)
    co = []
    D.fp_cg(A, b, 4, coeffs=co)
    assert co[0][2].all() and not co[1][2].any()       # frozen after the exact step
    assert D.lanczos_kappa(co)[0] == pytest.approx(1.0, abs=1e-14)


@pytest.mark.parametrize("variant", [0, 1])
def test_left_preconditioned_estimates_md_a(variant):
    rng = np.random.default_rng(3)
    A = _hpd(rng, 4, 8, 60.0)
    b = rng.standard_normal((4, 8, 2)) + 1j * rng.standard_normal((4, 8, 2))
    co = []
    D.fp_bj_cg(A, b, 8, 4, D.schedule("fp64", variant=variant), coeffs=co)
    M, _ = D.bj_inverse(A, 4)
    ev = np.sort(np.linalg.eigvals(M @ A).real, axis=-1)    # similar to A_bar: real, positive
    np.testing.assert_allclose(D.lanczos_kappa(co), ev[:, -1] / ev[:, 0], rtol=1e-7)


def test_symmetric_form_estimates_a_bar():
    rng = np.random.default_rng(4)
    A = _hpd(rng, 4, 8, 60.0)
    b = rng.standard_normal((4, 8, 2)) + 1j * rng.standard_normal((4, 8, 2))
    co = []
    x, broken, T, Abar = D.fp_bj_cg_split(A, b, 8, 4, D.schedule("fp64", variant=2), coeffs=co)
    np.testing.assert_allclose(D.lanczos_kappa(co), _kappa(T @ A @ np.conj(np.swapaxes(T, -1, -2))), rtol=1e-7)


def test_detect_records_the_first_solve():
    rng = np.random.default_rng(5)
    B, Nbs, K, R = 3, 24, 8, 4
    H = (rng.standard_normal((B, Nbs, K)) + 1j * rng.standard_normal((B, Nbs, K))) / np.sqrt(2 * Nbs)
    Y = rng.standard_normal((B, Nbs, R)) + 1j * rng.standard_normal((B, Nbs, R))
    s2 = np.full(B, 0.05)
    co = []
    D.detect(H, Y, s2, 16, K, 0, D.FP64, coeffs=co)
    A = np.conj(np.swapaxes(H, -1, -2)) @ H + 0.05 * np.eye(K)
    np.testing.assert_allclose(D.lanczos_kappa(co), _kappa(A), rtol=1e-8)
    assert len(co) == K
