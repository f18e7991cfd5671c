"""Pins of the oracle's detector: Gram / matched filter, Alg. 1-3, eq. pre_BJ,
the emulated matrix products, refresh, refinement, breakdown rules, slicer.

Each test checks the oracle against something independent of its own code:
exact rational arithmetic, closed forms, library solvers, element-by-element
loops with torch's rounding casts, or brute force over small inputs."""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
import torch

import workload as W
from oracle import detect as D


# ---------------------------------------------------------------- helpers
class GQ:
    """Exact Gaussian rational a + i b (a, b Fractions)."""
    __slots__ = ("re", "im")

    def __init__(self, re, im=0):
        self.re = Fraction(re)
        self.im = Fraction(im)

    def _c(o):
        return o if isinstance(o, GQ) else GQ(o)

    def __add__(s, o):
        if isinstance(o, np.ndarray):
            return NotImplemented
        o = GQ._c(o); return GQ(s.re + o.re, s.im + o.im)
    __radd__ = __add__

    def __sub__(s, o):
        if isinstance(o, np.ndarray):
            return NotImplemented
        o = GQ._c(o); return GQ(s.re - o.re, s.im - o.im)

    def __rsub__(s, o):
        return GQ._c(o) - s

    def __neg__(s):
        return GQ(-s.re, -s.im)

    def __mul__(s, o):
        if isinstance(o, np.ndarray):
            return NotImplemented
        o = GQ._c(o); return GQ(s.re * o.re - s.im * o.im, s.re * o.im + s.im * o.re)
    __rmul__ = __mul__

    def __truediv__(s, o):
        if isinstance(o, np.ndarray):
            return NotImplemented
        o = GQ._c(o); d = o.re * o.re + o.im * o.im
        return GQ((s.re * o.re + s.im * o.im) / d, (s.im * o.re - s.re * o.im) / d)

    def __rtruediv__(s, o):
        return GQ._c(o) / s

    def conjugate(s):
        return GQ(s.re, -s.im)

    @property
    def real(s):
        return s.re

    def __eq__(s, o):
        o = GQ._c(o); return s.re == o.re and s.im == o.im

    def __hash__(s):
        return hash((s.re, s.im))


def gq_array(re, im):
    out = np.empty(re.shape, dtype=object)
    for idx in np.ndindex(re.shape):
        out[idx] = GQ(int(re[idx]), int(im[idx]))
    return out


def exact_solve(A, b):
    """Gauss-Jordan over exact numbers (independent of the oracle)."""
    n = A.shape[0]
    M = np.concatenate([A.copy(), b.copy()], axis=1)
    for k in range(n):
        piv = next(i for i in range(k, n) if M[i, k] != 0)
        M[[k, piv]] = M[[piv, k]]
        M[k] = M[k] / M[k, k]
        for i in range(n):
            if i != k and M[i, k] != 0:
                M[i] = M[i] - M[i, k] * M[k]
    return M[:, n:]


def rand_hpd_int(n, seed):
    rng = np.random.default_rng(seed)
    re = rng.integers(-3, 4, (n + 2, n))
    im = rng.integers(-3, 4, (n + 2, n))
    H = gq_array(re, im)
    A = np.conj(H.T) @ H
    for i in range(n):
        A[i, i] = A[i, i] + 1
    return A


def small_wl(B=6, Nbs=32, K=8, R=3, q=16, snr=15.0, zeta=0.5, seed=0):
    return W.draw(B, Nbs, K, R, q, snr, zeta, zeta, seed=seed)


# ---------------------------------------------------------------- Gram / LMMSE
def test_gram_matches_elementwise_loop():
    wl = small_wl(B=2, Nbs=5, K=3, R=2)
    A, b = D.gram(wl.H, wl.Y, wl.sigma2)
    for c in range(2):
        for i in range(3):
            for j in range(3):
                ref = sum(np.conj(wl.H[c, m, i]) * wl.H[c, m, j] for m in range(5)) + (wl.sigma2[c] if i == j else 0)
                assert abs(A[c, i, j] - ref) < 1e-14
            for n in range(2):
                ref = sum(np.conj(wl.H[c, m, i]) * wl.Y[c, m, n] for m in range(5))
                assert abs(b[c, i, n] - ref) < 1e-14


def test_gram_is_hermitian_pd():
    wl = small_wl(B=20, Nbs=16, K=8)
    A, _ = D.gram(wl.H, wl.Y, wl.sigma2)
    assert np.array_equal(A, np.conj(np.swapaxes(A, -1, -2)))  # exactly Hermitian
    assert np.all(np.linalg.eigvalsh(A) > 0)


def test_lmmse_matches_library_solve():
    wl = small_wl(B=10, Nbs=24, K=8, R=4)
    A, b = D.gram(wl.H, wl.Y, wl.sigma2)
    x = D.lmmse(A, b)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-12)
    for c in range(10):
        assert np.allclose(x[c], sla.cho_solve(sla.cho_factor(A[c]), b[c]), rtol=0, atol=1e-12)


# ---------------------------------------------------------------- exact arithmetic
@pytest.mark.parametrize("n,seed", [(3, 1), (4, 2), (5, 3)])
def test_alg1_and_alg2_terminate_exactly_in_n_steps(n, seed):
    """Exact CG reaches x = A^{-1} b (and r = 0) in at most n steps."""
    A = rand_hpd_int(n, seed)
    rng = np.random.default_rng(seed + 10)
    b = gq_array(rng.integers(-5, 6, (n, 2)), rng.integers(-5, 6, (n, 2)))
    xs = exact_solve(A, b)
    x1 = D.cg_alg1(A[None], b[None], n)[0]
    assert all(x1[i, j] == xs[i, j] for i in range(n) for j in range(2))
    trace = []
    x2, broken = D.fp_cg(A[None], b[None], n, trace=trace)
    assert all(x2[0, i, j] == xs[i, j] for i in range(n) for j in range(2))
    _, r_last = trace[-1]
    assert all(v == 0 for v in r_last.ravel())
    assert not broken.any()


def test_alg3_exact_terminates_and_block_solution():
    n, L = 4, 2
    A = rand_hpd_int(n, 5)
    b = gq_array(np.array([[1], [2], [-1], [3]]), np.array([[0], [1], [2], [-2]]))
    M = np.zeros((n, n), dtype=object)
    M[...] = GQ(0)
    for j in range(n // L):
        sl = slice(j * L, (j + 1) * L)
        eye = np.empty((L, L), dtype=object)
        for i in range(L):
            for k in range(L):
                eye[i, k] = GQ(1 if i == k else 0)
        M[sl, sl] = exact_solve(A[sl, sl], eye)
    xs = exact_solve(A, b)
    for variant in (0, 1):
        x, _ = D.fp_bj_cg(A[None], b[None], n, L, D.Schedule(variant=variant), M=M[None])
        assert all(x[0, i, 0] == xs[i, 0] for i in range(n))


# ---------------------------------------------------------------- fp64 properties
def test_identity_scaled_converges_in_one_step():
    c = 3.7
    A = np.eye(6, dtype=np.complex128)[None] * c
    rng = np.random.default_rng(0)
    b = (rng.standard_normal((1, 6, 3)) + 1j * rng.standard_normal((1, 6, 3)))
    x, _ = D.fp_cg(A, b, 1)
    assert np.allclose(x, b / c, rtol=1e-15, atol=0)


def test_k_distinct_eigenvalues_converge_in_k_steps():
    rng = np.random.default_rng(1)
    n, k = 12, 3
    q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.repeat([1.0, 4.0, 9.0], n // k)
    A = (q * lam) @ q.conj().T
    A = 0.5 * (A + A.conj().T)
    b = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    xs = np.linalg.solve(A, b)
    x_k, _ = D.fp_cg(A[None], b[None], k)
    x_km1, _ = D.fp_cg(A[None], b[None], k - 1)
    assert np.linalg.norm(x_k[0] - xs) / np.linalg.norm(xs) < 1e-12
    assert np.linalg.norm(x_km1[0] - xs) / np.linalg.norm(xs) > 1e-3


def test_fp64_cg_with_K_iterations_matches_cholesky():
    wl = W.draw(50, 64, 8, 1, 16, 10.0, 0.0, 0.0, seed=11, normalization="unit")
    A, b = D.gram(wl.H, wl.Y, wl.sigma2)
    assert np.max(np.linalg.cond(A)) < 100
    x, _ = D.fp_cg(A, b, 8)
    xs = D.lmmse(A, b)
    rel = np.linalg.norm(x - xs, axis=-2) / np.linalg.norm(xs, axis=-2)
    assert np.max(rel) < 1e-12


def test_alg1_alg2_agree_and_residuals_orthogonal():
    wl = small_wl(B=8, Nbs=64, K=16, R=2, zeta=0.3)
    A, b = D.gram(wl.H, wl.Y, wl.sigma2)
    x1 = D.cg_alg1(A, b, 6)
    trace = []
    x2, _ = D.fp_cg(A, b, 6, trace=trace)
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x2) < 1e-12
    rs = [b] + [r for _, r in trace]
    for i in range(len(rs)):
        for j in range(i):
            ip = np.abs(np.sum(np.conj(rs[i]) * rs[j], axis=-2))
            nrm = np.linalg.norm(rs[i], axis=-2) * np.linalg.norm(rs[j], axis=-2)
            assert np.max(ip / nrm) < 1e-9


def test_alg3_variants_agree_and_match_symmetric_preconditioning():
    """Left-preconditioned Alg. 3 and CG on C^{-1} A C^{-H} give the same iterates."""
    wl = small_wl(B=5, Nbs=64, K=16, R=2, zeta=0.7)
    A, b = D.gram(wl.H, wl.Y, wl.sigma2)
    L = 4
    x0, _ = D.fp_bj_cg(A, b, 7, L, D.Schedule(variant=0))
    x1, _ = D.fp_bj_cg(A, b, 7, L, D.Schedule(variant=1))
    assert np.linalg.norm(x0 - x1) / np.linalg.norm(x0) < 1e-12
    C = np.zeros_like(A)
    for j in range(16 // L):
        sl = slice(j * L, (j + 1) * L)
        C[:, sl, sl] = np.linalg.cholesky(A[:, sl, sl])
    Ci = np.linalg.inv(C)
    Abar = Ci @ A @ np.conj(np.swapaxes(Ci, -1, -2))
    xbar = D.cg_alg1(Abar, Ci @ b, 7)
    x_sym = np.conj(np.swapaxes(Ci, -1, -2)) @ xbar
    assert np.linalg.norm(x0 - x_sym) / np.linalg.norm(x0) < 1e-11


def test_alg3_block_diagonal_gram_is_solved_in_one_step():
    """App. D: under Assumption 2 with L >= N_UE, the preconditioned matrix is I."""
    rng = np.random.default_rng(4)
    K, L, nue = 16, 8, 4
    blocks = []
    for u in range(K // nue):
        h = rng.standard_normal((64, nue)) + 1j * rng.standard_normal((64, nue))
        blocks.append(h.conj().T @ h / 64 + 0.1 * np.eye(nue))
    A = sla.block_diag(*blocks)[None]
    b = rng.standard_normal((1, K, 3)) + 1j * rng.standard_normal((1, K, 3))
    x, _ = D.fp_bj_cg(A, b, 1, L)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) / np.linalg.norm(x) < 1e-12
    # and with a single block (L = K), M_d = A^{-1}: one step for any A
    wl = small_wl(B=2, Nbs=32, K=8, R=2, zeta=0.6)
    A2, b2 = D.gram(wl.H, wl.Y, wl.sigma2)
    x2, _ = D.fp_bj_cg(A2, b2, 1, 8)
    assert np.linalg.norm(x2 - D.lmmse(A2, b2)) / np.linalg.norm(x2) < 1e-12


def test_bj_inverse_blocks_match_library_inverse():
    wl = small_wl(B=4, Nbs=64, K=16, R=1)
    A, _ = D.gram(wl.H, wl.Y, wl.sigma2)
    M, not_pd = D.bj_inverse(A, 4)
    assert not not_pd.any()
    for j in range(4):
        sl = slice(4 * j, 4 * j + 4)
        assert np.allclose(M[:, sl, sl], np.linalg.inv(A[:, sl, sl]), rtol=0, atol=1e-12)
    off = M.copy()
    for j in range(4):
        off[:, 4 * j:4 * j + 4, 4 * j:4 * j + 4] = 0
    assert np.all(off == 0)
    # M_d A has identity diagonal blocks
    MA = M @ A
    for j in range(4):
        sl = slice(4 * j, 4 * j + 4)
        assert np.allclose(MA[:, sl, sl], np.eye(4), atol=1e-12)


def test_bj_inverse_not_pd_falls_back_to_diagonal():
    A = np.array([[[1.0, 2.0], [2.0, 1.0]]], dtype=np.complex128)   # indefinite
    M, not_pd = D.bj_inverse(A, 2)
    assert not_pd[0]
    assert np.allclose(M[0], np.diag([1.0, 1.0]))


# ---------------------------------------------------------------- emulated schedules
def _bf16(v):
    return float(torch.tensor([v], dtype=torch.float32).to(torch.bfloat16).to(torch.float64))


def test_emulated_matvec_matches_elementwise_reference():
    """w_i = fl32( sum_k bf16(A_ik) bf16(p_k) ) computed exactly with fsum and torch casts."""
    rng = np.random.default_rng(5)
    n = 6
    A = (rng.standard_normal((1, n, n)) + 1j * rng.standard_normal((1, n, n))).astype(np.complex64).astype(np.complex128)
    p = (rng.standard_normal((1, n, 2)) + 1j * rng.standard_normal((1, n, 2))).astype(np.complex64).astype(np.complex128)
    w = D.MatVec(A, D.BF16)(p)
    for i in range(n):
        for c in range(2):
            re_terms, im_terms = [], []
            for k in range(n):
                ar, ai = _bf16(A[0, i, k].real), _bf16(A[0, i, k].imag)
                pr, pi = _bf16(p[0, k, c].real), _bf16(p[0, k, c].imag)
                re_terms += [ar * pr, -ai * pi]
                im_terms += [ar * pi, ai * pr]
            wr = float(np.float32(math.fsum(re_terms)))
            wi = float(np.float32(math.fsum(im_terms)))
            assert w[0, i, c].real == wr and w[0, i, c].imag == wi


def test_emulated_fp8_matvec_scales():
    rng = np.random.default_rng(6)
    n = 5
    A = (rng.standard_normal((1, n, n)) * 3 + 1j * rng.standard_normal((1, n, n))).astype(np.complex64).astype(np.complex128)
    p = (rng.standard_normal((1, n, 1)) * 1e-3 + 1j * rng.standard_normal((1, n, 1)) * 1e-3)
    w = D.MatVec(A, D.FP8)(p)
    e4 = lambda v: float(torch.tensor([v], dtype=torch.float64).to(torch.float32).to(torch.float8_e4m3fn).to(torch.float64))
    amaxA = max(np.max(np.abs(A.real)), np.max(np.abs(A.imag)))
    amaxP = max(np.max(np.abs(p.real)), np.max(np.abs(p.imag)))
    sA = 2.0 ** math.floor(math.log2(448 / amaxA))
    sP = 2.0 ** math.floor(math.log2(448 / amaxP))
    for i in range(n):
        t_re, t_im = [], []
        for k in range(n):
            ar, ai = e4(A[0, i, k].real * sA), e4(A[0, i, k].imag * sA)
            pr, pi = e4(float(np.float32(p[0, k, 0].real * sP))), e4(float(np.float32(p[0, k, 0].imag * sP)))
            t_re += [ar * pr, -ai * pi]
            t_im += [ar * pi, ai * pr]
        assert w[0, i, 0].real == float(np.float32(math.fsum(t_re))) / (sA * sP)
        assert w[0, i, 0].imag == float(np.float32(math.fsum(t_im))) / (sA * sP)


def test_emulated_gram_matches_elementwise_reference():
    wl = small_wl(B=1, Nbs=7, K=3, R=2)
    H = wl.H.astype(np.complex64).astype(np.complex128)
    Y = wl.Y.astype(np.complex64).astype(np.complex128)
    A, b = D.gram(H, Y, wl.sigma2, D.BF16)
    f32 = lambda v: float(np.float32(v))
    for i in range(3):
        for j in range(3):
            tr, ti = [], []
            for m in range(7):
                hr_i, hi_i = _bf16(H[0, m, i].real), _bf16(H[0, m, i].imag)
                hr_j, hi_j = _bf16(H[0, m, j].real), _bf16(H[0, m, j].imag)
                tr += [hr_i * hr_j, hi_i * hi_j]
                ti += [hr_i * hi_j, -hi_i * hr_j]
            are = f32(math.fsum(tr))
            if i == j:
                are = f32(are + f32(wl.sigma2[0]))
            assert A[0, i, j].real == are and A[0, i, j].imag == f32(math.fsum(ti))


def test_schedule_fma_vs_two_roundings_differ_but_both_bounded():
    # well-conditioned (zeta = 0): fp32 iterates stay within a few u_32 of fp64
    wl = small_wl(B=4, Nbs=64, K=16, R=2, zeta=0.0)
    A, b = D.gram(wl.H, wl.Y, wl.sigma2, D.FP32)
    x1, _ = D.fp_cg(A, b, 10, D.FP32)
    x2, _ = D.fp_cg(A, b, 10, D.schedule("fp32", fma=False))
    xs, _ = D.fp_cg(A, b, 10)
    assert not np.array_equal(x1, x2)
    for x in (x1, x2):
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-6


def test_remark1_ip_precision_does_not_move_attainable_accuracy():
    """Remark 1 / Sec. V-B: bf16 inner products leave the residual gap near the
    fp64 level, bf16 matrix-vector products raise it by orders of magnitude."""
    from oracle import theory as T
    wl = W.draw(40, 256, 32, 1, 16, 20.0, 0.5, 0.5, seed=3)
    A, b = D.gram(wl.H, wl.Y, wl.sigma2)
    xs = D.lmmse(A, b)

    def gap(s):
        tr = []
        D.fp_cg(A, b, 20, s, trace=tr)
        x, r = tr[-1]
        return np.median(T.residual_gap(A, b, x, r, xs))

    g64 = gap(D.paper_schedule())
    gip = gap(D.paper_schedule(u_ip="bf16"))
    gmv = gap(D.paper_schedule(u_mv="bf16"))
    assert gip < 1e3 * g64 + 1e-13
    assert gmv > 1e4 * max(gip, g64)


def test_refresh_reduces_error_floor_of_low_precision_mv():
    wl = W.draw(30, 256, 32, 2, 16, 25.0, 0.8, 0.8, seed=8)
    A, b = D.gram(wl.H, wl.Y, wl.sigma2)
    xs = D.lmmse(A, b)
    r0 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 40, 8, D.FP16)
    r1 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 40, 8, D.schedule("fp16", refresh_every=4))
    e0 = np.linalg.norm(r0.xhat - xs) / np.linalg.norm(xs)
    e1 = np.linalg.norm(r1.xhat - xs) / np.linalg.norm(xs)
    assert e1 < 0.3 * e0


def test_refinement_reaches_fp32_level_with_fp8_operands():
    wl = W.draw(20, 64, 8, 2, 16, 25.0, 0.3, 0.3, seed=9)
    A, b = D.gram(wl.H, wl.Y, wl.sigma2)
    xs = D.lmmse(A, b)
    r0 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 8, 4, D.FP8)
    r2 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 8, 4, D.schedule("e4m3", refine_steps=3))
    e0 = np.linalg.norm(r0.xhat - xs) / np.linalg.norm(xs)
    e2 = np.linalg.norm(r2.xhat - xs) / np.linalg.norm(xs)
    assert e2 < 1e-2 * e0


# ---------------------------------------------------------------- guard / flags
def test_zero_input_breaks_down_to_zero_and_flags():
    wl = small_wl(B=3, Nbs=16, K=4, R=2)
    Y = wl.Y.copy()
    Y[1] = 0
    r = D.detect(wl.H, Y, wl.sigma2, 16, 4, 0, D.FP32)
    assert np.all(r.xhat[1] == 0)
    assert r.flags[1] & D.FLAG_BREAKDOWN
    assert not (r.flags[0] & D.FLAG_BREAKDOWN)


def test_nonfinite_channel_is_isolated():
    wl = small_wl(B=4, Nbs=16, K=4, R=2)
    H = wl.H.copy()
    H[2, 3, 1] = np.nan
    r = D.detect(H, wl.Y, wl.sigma2, 16, 4, 2, D.BF16)
    ref = D.detect(wl.H[[0, 1, 3]], wl.Y[[0, 1, 3]], wl.sigma2[[0, 1, 3]], 16, 4, 2, D.BF16)
    assert r.flags[2] & D.FLAG_NONFINITE
    assert np.all(r.xhat[2] == 0)
    assert np.array_equal(r.xhat[[0, 1, 3]], ref.xhat)
    assert np.array_equal(r.flags[[0, 1, 3]], ref.flags)


# ---------------------------------------------------------------- slicer
@pytest.mark.parametrize("q", [4, 16, 64, 256])
def test_slicer_recovers_points_and_matches_brute_force(q):
    labels = np.arange(q)
    pts = W.qam_points(labels, q)
    for work in ("fp32", "fp64"):
        assert np.array_equal(D.slice_qam(pts, q, work), labels)
    rng = np.random.default_rng(q)
    z = (rng.uniform(-1.6, 1.6, 5000) + 1j * rng.uniform(-1.6, 1.6, 5000))
    d = np.abs(z[:, None] - pts[None, :])
    best = np.argmin(d, axis=1)
    srt = np.sort(d, axis=1)
    clear = srt[:, 1] - srt[:, 0] > 1e-9
    assert np.array_equal(D.slice_qam(z, q)[clear], labels[best][clear])


@pytest.mark.parametrize("q", [16, 64, 256])
def test_gray_neighbours_differ_in_one_bit(q):
    m = int(math.sqrt(q))
    labels = np.arange(q)
    pts = W.qam_points(labels, q)
    nu = math.sqrt(2 * (q - 1) / 3)
    step = 2 / nu
    for ell, p in zip(labels, pts):
        for dz in (step, 1j * step):
            nb = p + dz
            if abs(nb.real) < m / nu and abs(nb.imag) < m / nu:
                lab = D.slice_qam(np.array([nb]), q)[0]
                assert bin(int(lab) ^ int(ell)).count("1") == 1


def test_slicer_tie_goes_to_upper_level():
    q = 16
    nu = math.sqrt(2 * (q - 1) / 3)
    # boundary between levels -1/nu and +1/nu is 0; between 1/nu and 3/nu is 2/nu
    z = np.array([0.0 + 0.0j, 2.0 / nu + 0j])
    lab = D.slice_qam(z, q, "fp64")
    up = D.slice_qam(np.array([1 / nu + 0j, 3 / nu + 0j]), q, "fp64")
    assert lab[0] >> 2 == up[0] >> 2 and lab[1] >> 2 == up[1] >> 2


def test_noise_free_high_snr_exact_recovery():
    wl = W.draw(20, 64, 8, 4, 64, 60.0, 0.2, 0.2, seed=12, noiseless=True)
    r = D.detect(wl.H, wl.Y, wl.sigma2, 64, 8, 0, D.FP64)
    assert np.array_equal(r.labels, wl.labels)
    r = D.detect(wl.H, wl.Y, wl.sigma2, 64, 8, 4, D.FP32)
    assert np.array_equal(r.labels, wl.labels)


def test_bit_errors_brute_force():
    rng = np.random.default_rng(0)
    a = rng.integers(0, 256, 1000)
    b = rng.integers(0, 256, 1000)
    assert D.bit_errors(a, b) == sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b))


# ---------------------------------------------------------------- sequential accumulation order
def test_sequential_matvec_is_an_ordered_fma_chain():
    """accum='sequential': each output is the fp32 fused multiply-add chain over k."""
    rng = np.random.default_rng(8)
    n = 5
    A = (rng.standard_normal((1, n, n)) + 1j * rng.standard_normal((1, n, n))).astype(np.complex64).astype(np.complex128)
    p = (rng.standard_normal((1, n, 2)) + 1j * rng.standard_normal((1, n, 2))).astype(np.complex64).astype(np.complex128)
    w = D.MatVec(A, D.schedule("bf16", accum="sequential"))(p)
    f32 = lambda v: float(np.float32(v))
    for i in range(n):
        for c in range(2):
            wr = wi = 0.0
            for k in range(n):
                ar, ai = _bf16(A[0, i, k].real), _bf16(A[0, i, k].imag)
                pr, pi = _bf16(p[0, k, c].real), _bf16(p[0, k, c].imag)
                wr = f32(ar * pr + wr)
                wr = f32(-ai * pi + wr)
                wi = f32(ai * pr + wi)
                wi = f32(ar * pi + wi)
            assert w[0, i, c].real == wr and w[0, i, c].imag == wi


def test_sequential_order_agrees_with_exact_order_when_well_conditioned():
    wl = small_wl(B=4, Nbs=64, K=16, R=2, zeta=0.0)
    r1 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 6, 4, D.FP64)
    r2 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 6, 4, D.schedule("fp64", accum="sequential"))
    assert np.linalg.norm(r1.xhat - r2.xhat) / np.linalg.norm(r1.xhat) < 1e-13
    r3 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 6, 4, D.FP32)
    r4 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 6, 4, D.schedule("fp32", accum="sequential"))
    assert 0 < np.linalg.norm(r3.xhat - r4.xhat) / np.linalg.norm(r3.xhat) < 1e-5
    A, _ = D.gram(wl.H, wl.Y, wl.sigma2, D.schedule("fp32", accum="sequential"))
    assert np.array_equal(A, np.conj(np.swapaxes(A, -1, -2)))


def test_split_form_matches_alg3_in_fp64():
    """Left-preconditioned Alg. 3 and its symmetric form give the same iterates."""
    for zeta, L in ((0.5, 4), (0.8, 8)):
        wl = small_wl(B=5, Nbs=64, K=16, R=3, zeta=zeta)
        r0 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 7, L, D.Schedule(variant=0))
        r2 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 7, L, D.Schedule(variant=2))
        assert np.linalg.norm(r0.xhat - r2.xhat) / np.linalg.norm(r0.xhat) < 1e-11


def test_split_system_is_identity_on_diagonal_blocks_and_hermitian():
    wl = small_wl(B=3, Nbs=64, K=16, R=1, zeta=0.7)
    A, _ = D.gram(wl.H, wl.Y, wl.sigma2)
    T, bad = D.bj_factor(A, 4)
    assert not bad.any()
    Ab = D.split_system(A, T)
    assert np.array_equal(Ab, np.conj(np.swapaxes(Ab, -1, -2)))
    for j in range(4):
        sl = slice(4 * j, 4 * j + 4)
        assert np.allclose(Ab[:, sl, sl], np.eye(4), atol=1e-12)
    M, _ = D.bj_inverse(A, 4)
    assert np.allclose(np.conj(np.swapaxes(T, -1, -2)) @ T, M, atol=1e-12)   # M_d = T^H T
    # T is block lower triangular
    for j in range(4):
        sl = slice(4 * j, 4 * j + 4)
        assert np.all(np.triu(T[:, sl, sl], 1) == 0)


def test_split_form_refinement_and_low_precision():
    wl = W.draw(6, 64, 16, 2, 16, 25.0, 0.6, 0.6, seed=31)
    A, b = D.gram(wl.H, wl.Y, wl.sigma2)
    xs = D.lmmse(A, b)
    r = D.detect(wl.H, wl.Y, wl.sigma2, 16, 10, 4, D.schedule("fp16", variant=2, refine_steps=2))
    assert np.linalg.norm(r.xhat - xs) / np.linalg.norm(xs) < 1e-5
    r1 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 10, 4, D.schedule("fp16", variant=2, refresh_every=3))
    r0 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 10, 4, D.schedule("fp16", variant=0, refresh_every=3))
    assert np.linalg.norm(r1.xhat - xs) / np.linalg.norm(xs) < 2 * np.linalg.norm(r0.xhat - xs) / np.linalg.norm(xs) + 1e-4


# ---------------------------------------------------------------- a kept block-Jacobi factor
def test_given_factor_of_this_channel_reproduces_the_factorisation():
    """T_given = the factor of this A: the symmetric form is bitwise the
    default path (the same T), the left form equals it to FP64 rounding
    (M_d formed as T^H T instead of C^{-H} C^{-1})."""
    wl = small_wl(B=4, Nbs=64, K=16, R=3, zeta=0.6, seed=11)
    A, _ = D.gram(wl.H, wl.Y, wl.sigma2)
    T, _ = D.bj_factor(A, 4)
    r2 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 6, 4, D.Schedule(variant=2))
    g2 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 6, 4, D.Schedule(variant=2), T_given=T)
    assert np.array_equal(r2.xhat, g2.xhat) and np.array_equal(r2.labels, g2.labels)
    r1 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 6, 4, D.Schedule(variant=1))
    g1 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 6, 4, D.Schedule(variant=1), T_given=T)
    assert np.linalg.norm(r1.xhat - g1.xhat) / np.linalg.norm(r1.xhat) < 1e-12


def test_identity_factor_is_plain_cg_bitwise():
    """T = I: A_bar = A exactly, b_bar = b, x = x_bar, so the symmetric form is
    Alg. 2 on A, bit for bit."""
    wl = small_wl(B=3, Nbs=32, K=8, R=2, zeta=0.5, seed=12)
    eye = np.broadcast_to(np.eye(8, dtype=np.complex128), (3, 8, 8)).copy()
    for name in ("fp64", "fp16"):
        s0 = D.schedule(name)
        s2 = D.schedule(name, variant=2)
        r0 = D.detect(wl.H, wl.Y, wl.sigma2, 16, 5, 0, s0)
        g = D.detect(wl.H, wl.Y, wl.sigma2, 16, 5, 4, s2, T_given=eye)
        assert np.array_equal(r0.xhat, g.xhat), name


def test_stale_factor_still_converges_to_lmmse():
    """Any Hermitian positive definite preconditioner leaves the CG solution
    unchanged: with the factor of an earlier, different channel realisation
    (Gauss-Markov step), FP64 PCG at I = 3K reaches the Cholesky LMMSE solution
    of the new channel, in both forms."""
    wls = W.gauss_markov(3, 64, 16, 2, 16, 20.0, 0.6, 0.6, steps=2, fd_hz=1000.0, seed=13)
    A0, _ = D.gram(wls[0].H, wls[0].Y, wls[0].sigma2)
    T0, _ = D.bj_factor(A0, 4)
    A1, b1 = D.gram(wls[1].H, wls[1].Y, wls[1].sigma2)
    xs = D.lmmse(A1, b1)
    for v in (1, 2):
        g = D.detect(wls[1].H, wls[1].Y, wls[1].sigma2, 16, 48, 4, D.Schedule(variant=v), T_given=T0)
        assert np.max(np.linalg.norm(g.xhat - xs, axis=-2) / np.linalg.norm(xs, axis=-2)) < 1e-10
