"""Seeded synthetic inputs for massive-MIMO uplink detection.

This module only *draws inputs*: correlated Rayleigh channels, uniformly
distributed Gray-mapped QAM symbols and AWGN.  It contains none of the
detector's arithmetic (no Gram matrix, no solver, no slicer), so both the
CPU oracle and the GPU path can consume the same seeded draws without
sharing any method code.

Signal model (paper, Sec. II): y = H x + n, with the Kronecker channel
H = sqrt(R_r) Omega sqrt(R_t) (eq. channel_model), Omega i.i.d. CN(0, 1/M),
and exponential correlation r_ij = zeta^(j-i) for i <= j, r_ji = conj(r_ij).

Readings of points the paper leaves open:
  * sqrt(R) is the symmetric PSD principal square root (eigen-decomposition
    with eigenvalues clipped at zero); the proof of Theorem 3 uses V^T = V.
  * The transmit correlation R_t spans all K streams (eqs. 3-4).
  * SNR = Es * E||h_k||^2 / sigma^2 with unit-energy symbols (Es = 1).  With
    CN(0, 1/M) entries E||h_k||^2 = 1, so sigma^2 = 1/SNR; with CN(0, 1)
    entries sigma^2 = M/SNR.  The detector output is invariant to this
    normalisation.
  * QAM labels use an independent binary-reflected Gray code per axis, with
    the in-phase bits in the high half of the label.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "exp_corr",
    "psd_sqrt",
    "qam_points",
    "Workload",
    "draw",
    "sigma2_from_snr_db",
    "imperfect_csi",
    "gauss_markov",
    "geometry",
    "CONFIGS",
]


def exp_corr(n: int, zeta: float) -> np.ndarray:
    """Exponential correlation matrix (Sec. II): r_ij = zeta^(j-i), i <= j."""
    idx = np.arange(n)
    d = idx[None, :] - idx[:, None]
    r = np.power(complex(zeta), np.abs(d)).astype(np.complex128)
    # lower triangle is the conjugate of the upper one
    low = d < 0
    r[low] = np.conj(r[low])
    if zeta == 0:
        r = np.eye(n, dtype=np.complex128)
    return r


def psd_sqrt(r: np.ndarray) -> np.ndarray:
    """Hermitian PSD principal square root via eigh (eigenvalues clipped at 0)."""
    w, v = np.linalg.eigh(r)
    w = np.clip(w, 0.0, None)
    return (v * np.sqrt(w)[None, :]) @ v.conj().T


def _gray_inverse(g: np.ndarray) -> np.ndarray:
    n = g.copy()
    shift = 1
    while True:
        s = n >> shift
        if not np.any(s):
            break
        n ^= s
        shift <<= 1
    # one more pass is harmless; loop above terminates when all shifted bits are 0
    return n


def qam_points(labels: np.ndarray, q: int) -> np.ndarray:
    """Map Gray labels to unit-energy square-QAM points (generator side)."""
    m = int(round(math.sqrt(q)))
    if m * m != q or q < 4:
        raise ValueError(f"square QAM order required, got {q}")
    b = m.bit_length() - 1
    labels = np.asarray(labels, dtype=np.int64)
    ji = _gray_inverse(labels >> b)
    jq = _gray_inverse(labels & (m - 1))
    nu = math.sqrt(2.0 * (q - 1) / 3.0)
    return ((2 * ji - (m - 1)) + 1j * (2 * jq - (m - 1))) / nu


def sigma2_from_snr_db(snr_db: float, nbs: int, normalization: str = "paper") -> float:
    """Noise variance for a given SNR (dB) under the adopted SNR reading."""
    snr = 10.0 ** (snr_db / 10.0)
    gain = 1.0 if normalization == "paper" else float(nbs)
    return gain / snr


@dataclasses.dataclass
class Workload:
    H: np.ndarray          # (B, Nbs, K) complex128
    Y: np.ndarray          # (B, Nbs, R) complex128
    labels: np.ndarray     # (B, K, R) int64, transmitted Gray labels
    X: np.ndarray          # (B, K, R) complex128, transmitted symbols
    sigma2: np.ndarray     # (B,) float64
    q: int
    snr_db: np.ndarray     # (B,) float64
    H_true: np.ndarray = None   # the channel Y was drawn with, when H is only an estimate of it

    @property
    def shape(self):
        b, nbs, k = self.H.shape
        return b, nbs, k, self.Y.shape[2]


def draw(
    B: int,
    Nbs: int,
    K: int,
    R: int,
    q: int,
    snr_db,
    zeta_r: float = 0.0,
    zeta_t: float = 0.0,
    seed: int = 0,
    normalization: str = "paper",
    noiseless: bool = False,
    chunk: int = 2048,
) -> Workload:
    """Draw B independent channels with R received vectors each.

    ``snr_db`` may be a scalar or a length-B array; ``zeta_r``/``zeta_t`` are
    the BS- and user-side exponential correlation coefficients.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    var = 1.0 / Nbs if normalization == "paper" else 1.0
    sr = psd_sqrt(exp_corr(Nbs, zeta_r)) if zeta_r else None
    st = psd_sqrt(exp_corr(K, zeta_t)) if zeta_t else None
    H = np.empty((B, Nbs, K), dtype=np.complex128)
    for s in range(0, B, chunk):
        e = min(B, s + chunk)
        n = e - s
        om = (rng.standard_normal((n, Nbs, K)) + 1j * rng.standard_normal((n, Nbs, K))) * math.sqrt(var / 2.0)
        if sr is not None:
            om = np.matmul(sr[None], om)
        if st is not None:
            om = np.matmul(om, st[None])
        H[s:e] = om
    labels = rng.integers(0, q, size=(B, K, R), dtype=np.int64)
    X = qam_points(labels, q)
    snr = np.broadcast_to(np.asarray(snr_db, dtype=np.float64), (B,)).copy()
    sigma2 = np.array([sigma2_from_snr_db(s, Nbs, normalization) for s in snr]) if B else np.zeros(0)
    Y = np.matmul(H, X)
    if not noiseless:
        nz = (rng.standard_normal((B, Nbs, R)) + 1j * rng.standard_normal((B, Nbs, R)))
        Y = Y + nz * np.sqrt(sigma2 / 2.0)[:, None, None]
    return Workload(H=H, Y=Y, labels=labels, X=X, sigma2=sigma2, q=q, snr_db=snr)


# ---------------------------------------------------------------- robustness workloads
# (Sec. V, robustness to imperfect CSI, geometry-based and time-varying channels)

def imperfect_csi(wl: Workload, eps_db: float, seed: int = 0) -> Workload:
    """The workload seen through a channel estimate H_hat = H + dH: dH has
    i.i.d. CN(0, P / eps) entries, P the mean entry power of H and eps the
    channel-to-error power ratio (10^(eps_db/10)).  Y keeps the true channel
    (kept in ``H_true``); H becomes the estimate the detector uses."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = float(np.mean(np.abs(wl.H) ** 2))
    var = P / 10.0 ** (eps_db / 10.0)
    dH = (rng.standard_normal(wl.H.shape) + 1j * rng.standard_normal(wl.H.shape)) * math.sqrt(var / 2.0)
    return dataclasses.replace(wl, H=wl.H + dH, H_true=wl.H)


def gauss_markov(B: int, Nbs: int, K: int, R: int, q: int, snr_db: float, zeta_r: float, zeta_t: float,
                 steps: int, fd_hz: float, tau_s: float = 1.0 / 14000.0, seed: int = 0,
                 normalization: str = "paper") -> list:
    """First-order Gauss-Markov evolution H_i = rho H_{i-1} + sqrt(1 - rho^2) W_i
    with rho = J0(2 pi f_d tau) and W_i independent draws of the same Kronecker
    covariance; each step carries new symbols and noise.  tau defaults to one
    OFDM symbol at 15 kHz subcarrier spacing (a reading: the paper does not
    give it).  Returns the list of the steps' workloads."""
    from scipy.special import j0

    rho = float(j0(2.0 * math.pi * fd_hz * tau_s))
    out = [draw(B, Nbs, K, R, q, snr_db, zeta_r, zeta_t, seed=seed, normalization=normalization)]
    for i in range(1, steps):
        w = draw(B, Nbs, K, R, q, snr_db, zeta_r, zeta_t, seed=seed + 7919 * i, normalization=normalization)
        H = rho * out[-1].H + math.sqrt(max(0.0, 1.0 - rho * rho)) * w.H
        rng = np.random.Generator(np.random.PCG64(seed + 104729 * i))
        Y = np.matmul(H, w.X)
        nz = rng.standard_normal(Y.shape) + 1j * rng.standard_normal(Y.shape)
        Y = Y + nz * np.sqrt(w.sigma2 / 2.0)[:, None, None]
        out.append(dataclasses.replace(w, H=H, Y=Y))
    return out


def geometry(B: int, Nbs: int, K: int, R: int, q: int, snr_db, paths: int = 5, mu: float = 1.0, seed: int = 0) -> Workload:
    """Geometry-based multipath channel for single-antenna users: column k is
    sum_i alpha_i a(phi_i) over `paths` paths, the first (line of sight) with
    alpha ~ CN(0, 1), the others CN(0, 10^-mu), angles of arrival U(-pi, pi)
    at a half-wavelength uniform linear array, a(phi) = [e^{j pi n sin phi}] /
    sqrt(Nbs).  Readings: the base-station response is the array's column
    (the paper's a_t a_r^H written as the M x N_k matrix a_r a_t^H, a_t = 1 for
    one antenna); columns are scaled to E||h_k||^2 = 1 so the SNR reading of
    draw() applies (the scale does not change x_hat)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gain = np.sqrt(np.concatenate([[1.0], np.full(paths - 1, 10.0 ** (-mu))]))
    norm = 1.0 / math.sqrt(float(np.sum(gain ** 2)))
    n = np.arange(Nbs)
    H = np.zeros((B, Nbs, K), dtype=np.complex128)
    for p in range(paths):
        phi = rng.uniform(-math.pi, math.pi, size=(B, 1, K))
        a = np.exp(1j * math.pi * n[None, :, None] * np.sin(phi)) / math.sqrt(Nbs)
        alpha = (rng.standard_normal((B, 1, K)) + 1j * rng.standard_normal((B, 1, K))) * (gain[p] / math.sqrt(2.0))
        H += alpha * a
    H *= norm                                         # E||h_k||^2 = 1
    labels = rng.integers(0, q, size=(B, K, R), dtype=np.int64)
    X = qam_points(labels, q)
    snr = np.broadcast_to(np.asarray(snr_db, dtype=np.float64), (B,)).copy()
    sigma2 = np.array([sigma2_from_snr_db(s, Nbs, "paper") for s in snr])
    Y = np.matmul(H, X)
    nz = rng.standard_normal(Y.shape) + 1j * rng.standard_normal(Y.shape)
    Y = Y + nz * np.sqrt(sigma2 / 2.0)[:, None, None]
    return Workload(H=H, Y=Y, labels=labels, X=X, sigma2=sigma2, q=q, snr_db=snr)


# The five workloads the benchmarks and parity tests are built on
# (shapes, modulation, correlation, SNR, iteration counts).
CONFIGS = {
    "c1": dict(Nbs=64, K=8, R=1, B=1000, q=16, zeta=0.0, snr_db=10.0, normalization="unit"),
    "c2": dict(Nbs=128, K=32, R=14, B=16384, q=64, zeta=0.5, snr_db=20.0, normalization="paper"),
    "c3": dict(Nbs=256, K=64, R=14, B=8192, q=64, zeta=0.7, snr_db=15.0, normalization="paper"),
    "c4": dict(Nbs=512, K=128, R=14, B=2048, q=256, zeta=0.9, snr_db=25.0, normalization="paper"),
    # the paper's own simulation setup (Sec. V-A): M=256, N=32, 16-QAM, L=8
    "paper": dict(Nbs=256, K=32, R=1, B=4096, q=16, zeta=0.8, snr_db=20.0, normalization="paper"),
}
