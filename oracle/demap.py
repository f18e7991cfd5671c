"""Plain CPU oracle of soft-output (max-log LLR) demapping after the detector.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper evaluates its detector in a coded link (Sec. V, Fig. coding:
rate-1/2 convolutional code, Viterbi decoding, 16-QAM) without stating how
bits are handed to the decoder.  Readings taken here:

  * Post-detection model of the LMMSE estimate (eq. inversion with unit-energy
    symbols): x_hat_k = mu_k s_k + e_k, e_k of variance nu_k^2 = mu_k (1 - mu_k),
    with mu_k = (A^{-1} H^H H)_kk = 1 - sigma^2 (A^{-1})_kk.  The detector
    never forms A^{-1}; its block-Jacobi preconditioner M_d (eq. pre_BJ) holds
    the inverses of A's diagonal blocks, so mu_k = 1 - sigma^2 (M_d)_kk, with
    1 / A_kk where no preconditioner is used.  With one block (L = K) this is
    the exact LMMSE gain.
  * Max-log LLR of label bit b, positive when the bit is more likely 0:
    LLR_b = (min_{s: b(s)=1} |x_hat - mu s|^2 - min_{s: b(s)=0} |x_hat - mu s|^2) / nu^2,
    over the Q points of the unit-energy Gray square QAM the slicer uses;
    bits listed from the label's most significant bit.
  * Degenerate gains: mu is clamped to [0, 1] (NaN kept).  Where
    nu^2 = mu (1 - mu) is not positive (mu = 0: nothing received; mu = 1:
    zero-forcing, sigma^2 = 0, where the detector knows no noise level) the
    LLR is 0 where the two distances tie and +-inf otherwise.

Functions
  * constellation(q):       the Q points and their labels.
  * effective_gain(A, sigma2, L): mu_k from the Gram A (u_W) and eq. pre_BJ.
  * maxlog_llr(xhat, gain, q): the max-log LLRs, brute force over all Q points.
  * logmap_llr(xhat, gain, q): the exact LLRs of the same Gaussian model (the
    sum over points), used by the tests to pin the max-log values.
"""
from __future__ import annotations

import math

import numpy as np

from .detect import bj_inverse


def _gray(n):
    return n ^ (n >> 1)


def constellation(q: int):
    """(points (Q,) complex128, labels (Q,) int64) of unit-energy square Gray QAM:
    per axis level j in 0..m-1 at (2j - m + 1) / sqrt(2 (Q - 1) / 3), label
    (gray(j_I) << log2 m) | gray(j_Q)."""
    m = int(round(math.sqrt(q)))
    if m * m != q or m < 2 or m & (m - 1):
        raise ValueError("q must be 4, 16, 64 or 256")
    bits = m.bit_length() - 1
    nu = math.sqrt(2.0 * (q - 1) / 3.0)
    lev = (2.0 * np.arange(m) - (m - 1)) / nu
    ji, jq = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    pts = (lev[ji] + 1j * lev[jq]).ravel()
    labels = ((_gray(ji) << bits) | _gray(jq)).ravel().astype(np.int64)
    return pts, labels


def effective_gain(A, sigma2, L: int, work: str = "fp64"):
    """mu (B, K) = 1 - sigma^2 diag(M), M = M_d of eq. pre_BJ for L > 0 (the
    inverses of A's L x L diagonal blocks, with the diagonal fallback of a
    block that is not positive definite), and diag(A)^{-1} for L = 0."""
    A = np.asarray(A)
    s2 = np.asarray(sigma2, dtype=np.float64).reshape(-1, 1)
    M, _ = bj_inverse(A, L if L > 0 else 1, work)
    return 1.0 - s2 * np.real(np.diagonal(M, axis1=-2, axis2=-1))


def _gain_nu2(gain):
    g = np.asarray(gain, dtype=np.float64)
    with np.errstate(invalid="ignore"):
        g = np.where(g < 0, 0.0, np.where(g > 1, 1.0, g))
    return g, g * (1.0 - g)


def _bit_distances(xhat, gain, q):
    """(D0, D1): per label bit (most significant first) the smallest
    |x_hat - mu s|^2 over the points whose bit is 0 / 1; shapes (..., bits)."""
    pts, labels = constellation(q)
    nb = int(round(math.log2(q)))
    x = np.asarray(xhat, dtype=np.complex128)[..., None]
    g = np.asarray(gain, dtype=np.float64)[..., None]
    d = np.abs(x - g * pts) ** 2                              # (..., Q)
    D0 = np.empty(x.shape[:-1] + (nb,))
    D1 = np.empty(x.shape[:-1] + (nb,))
    for t in range(nb):
        bit = (labels >> (nb - 1 - t)) & 1
        D0[..., t] = np.min(d[..., bit == 0], axis=-1)
        D1[..., t] = np.min(d[..., bit == 1], axis=-1)
    return D0, D1


def maxlog_llr(xhat, gain, q: int):
    """Max-log LLRs, shape xhat.shape + (log2 q,), most significant label bit
    first.  gain broadcasts against xhat (e.g. (B, K, 1) for xhat (B, K, R))."""
    g, nu2 = _gain_nu2(gain)
    g = np.broadcast_to(g, np.shape(xhat))
    nu2 = np.broadcast_to(nu2, np.shape(xhat))[..., None]
    D0, D1 = _bit_distances(xhat, g, q)
    diff = D1 - D0
    with np.errstate(divide="ignore", invalid="ignore"):
        llr = np.where(nu2 > 0, diff / np.where(nu2 > 0, nu2, 1.0), np.sign(diff) * np.inf)
    llr = np.where(diff == 0, 0.0, llr)
    return np.where(np.isnan(nu2) | np.isnan(diff), np.nan, llr)


def logmap_llr(xhat, gain, q: int):
    """Exact LLRs of the model x_hat = mu s + e, e ~ CN(0, nu^2), uniform
    symbols: log of the summed likelihoods of the bit-0 points over those of
    the bit-1 points (nu^2 > 0 required)."""
    g, nu2 = _gain_nu2(gain)
    g = np.broadcast_to(g, np.shape(xhat))[..., None]
    nu2 = np.broadcast_to(nu2, np.shape(xhat))[..., None]
    pts, labels = constellation(q)
    nb = int(round(math.log2(q)))
    x = np.asarray(xhat, dtype=np.complex128)[..., None]
    e = -np.abs(x - g * pts) ** 2 / nu2                      # (..., Q)
    out = np.empty(np.shape(xhat) + (nb,))
    for t in range(nb):
        bit = (labels >> (nb - 1 - t)) & 1
        e0, e1 = e[..., bit == 0], e[..., bit == 1]
        m0 = np.max(e0, axis=-1, keepdims=True)
        m1 = np.max(e1, axis=-1, keepdims=True)
        l0 = m0[..., 0] + np.log(np.sum(np.exp(e0 - m0), axis=-1))
        l1 = m1[..., 0] + np.log(np.sum(np.exp(e1 - m1), axis=-1))
        out[..., t] = l0 - l1
    return out
