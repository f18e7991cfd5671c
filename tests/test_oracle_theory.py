"""Pins of the oracle's analysis helpers against the paper's printed numbers,
closed forms and Monte Carlo."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workload as W
from oracle import detect as D
from oracle import theory as T
from oracle.rounding import UNIT_ROUNDOFF

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


# ---------------------------------------------------------------- cost model
def _cases():
    N, L = 32, 8
    cg15, cg17, cg10 = T.cost_cg(N, 15), T.cost_cg(N, 17), T.cost_cg(N, 10)
    inv = T.cost_lmmse(N)
    fpcg17, fpcg21 = T.cost_cg(N, 17, "fp32"), T.cost_cg(N, 21, "fp32")
    bj10, bj13 = T.cost_bj_cg(N, L, 10, "fp16"), T.cost_bj_cg(N, L, 13, "fp16")
    return [
        T.reduction(fpcg17, cg15), T.reduction(fpcg17, inv), T.reduction(bj10, cg15), T.reduction(bj10, inv),
        T.reduction(bj10, cg10), T.reduction(T.cost_cg(N, 10, "fp16"), cg10),
        T.reduction(bj13, cg17), T.reduction(bj13, inv), T.reduction(fpcg21, cg17), T.reduction(fpcg21, inv),
    ]


def test_cost_model_reproduces_printed_percentages():
    got = _cases()
    for val, case in zip(got, GOLD["cost_model"]["cases"]):
        tol = case.get("tol", 0.05)
        assert abs(val - case["pct"]) <= tol, (case["what"], val)


def test_bj_setup_equals_two_cg_iterations():
    N, L = 32, 8
    assert T.cost_bj_setup(N, L) == GOLD["cost_model"]["bj_setup_in_cg_iterations"]["value"] * T.cost_cg(N, 1)


def test_example_1_demand():
    ex = GOLD["example_1"]
    flops = ex["iters"] * ex["N"] ** 2     # complex multiply count per subchannel
    assert flops == ex["flops_per_subchannel"]
    tflops = flops * ex["subcarriers"] / ex["slot_s"] / 1e12
    assert abs(tflops - ex["tflops_approx"]) < 1.5


# ---------------------------------------------------------------- heuristic
def test_gamma_and_bound_shape():
    assert T.gamma(10, 1e-3) == pytest.approx(0.01 / 0.99)
    assert T.gamma(10, 0.2) == math.inf
    b1 = T.attainable_bound(5, 32, 2.0**-24, 2.0**-11, 3.0)
    b2 = T.attainable_bound(5, 32, 2.0**-24, 2.0**-8, 3.0)
    assert b2 > 7 * b1   # dominated by the u_MV term (Remark 1)


def test_heuristic_threshold_of_the_paper():
    h = GOLD["heuristic"]
    # the printed threshold corresponds to E{kappa} ~ 17.3 at N = 32
    kappa_implied = (1.0 / (h["u_bound"] * h["N"] ** 1.5)) ** 2
    assert 15 < kappa_implied < 20
    wl = W.draw(300, h["M"], h["N"], 1, 16, h["snr_db"], h["zeta"], h["zeta"], seed=101)
    k = T.expected_kappa(wl.H, wl.sigma2)
    bound = T.heuristic_bound(h["N"], k)
    assert bound == pytest.approx(h["u_bound"], rel=0.15)
    assert T.select_format(h["N"], k, allow_fp8=False) == h["selected"]


def test_heuristic_picks_follow_the_paper():
    picks = GOLD["heuristic_picks"]
    N, L = 32, picks["L"]
    for z, fmt in picks["fpcg"].items():
        wl = W.draw(200, 256, N, 1, 16, 20.0, float(z), float(z), seed=7)
        assert T.select_format(N, T.expected_kappa(wl.H, wl.sigma2), allow_fp8=False) == fmt, z
    for z, fmt in picks["fpbjcg"].items():
        wl = W.draw(200, 256, N, 1, 16, 20.0, float(z), float(z), seed=8)
        kb = T.expected_kappa(wl.H, wl.sigma2, L)
        assert T.select_format(N, kb, allow_fp8=False) == fmt, z
        assert kb < T.expected_kappa(wl.H, wl.sigma2)    # Thm 5 direction


def test_select_format_order():
    assert T.select_format(4, 1.0) == "e4m3"
    assert T.select_format(4, 1.0, allow_fp8=False) == "fp16"
    assert T.select_format(1000, 1e6) == "fp64"
    assert T.select_format(32, 100.0) == "fp16"      # bound 5.5e-4 > u_fp16
    assert T.select_format(32, 1000.0) == "fp32"     # bound 1.7e-4


# ---------------------------------------------------------------- App. B moments
@pytest.mark.parametrize("M,zeta", [(2, 0.4), (3, 0.7), (64, 0.6), (256, 0.9)])
def test_gram_variance_closed_form_matches_finite_sum(M, zeta):
    s = sum((M - d) * zeta ** (2 * d) for d in range(1, M))
    direct = 1.0 / M + 2.0 / M**2 * s
    assert T.gram_entry_variance(M, zeta) == pytest.approx(direct, rel=1e-12)


def test_gram_moments_monte_carlo():
    """E{H^H H} = R_t and the off-diagonal variance of eq. var (independent of R_t)."""
    M, K, zr, zt = 64, 4, 0.6, 0.5
    wl = W.draw(20000, M, K, 1, 4, 10.0, zr, zt, seed=3)
    G = np.conj(np.swapaxes(wl.H, -1, -2)) @ wl.H
    Rt = W.exp_corr(K, zt)
    mean = G.mean(axis=0)
    var01 = np.mean(np.abs(G[:, 0, 1] - Rt[0, 1]) ** 2)
    se = math.sqrt(T.gram_entry_variance(M, zr) / 20000)
    assert np.max(np.abs(mean - Rt)) < 6 * se
    assert var01 == pytest.approx(T.gram_entry_variance(M, zr), rel=0.05)


# ---------------------------------------------------------------- Thm 2 / Thm 4 bound
@pytest.mark.parametrize("mv", ["fp16", "bf16", "fp32"])
def test_thm2_bound_holds_for_emulated_runs(mv):
    wl = W.draw(30, 256, 32, 2, 16, 20.0, 0.5, 0.5, seed=21)
    A, b = D.gram(wl.H, wl.Y, wl.sigma2)
    xs = D.lmmse(A, b)
    s = D.paper_schedule(u_mv=mv, u_ip="fp64", u_w="fp64")
    tr = []
    D.fp_cg(A, b, 25, s, trace=tr)
    u_mv = UNIT_ROUNDOFF[mv]
    norms = [np.linalg.norm(x, axis=-2) for x, _ in tr]
    nx = np.linalg.norm(xs, axis=-2)
    for i, (x, r) in enumerate(tr, start=1):
        theta = np.max(np.stack(norms[:i]), axis=0) / nx
        gap = T.residual_gap(A, b, x, r, xs)
        bound = np.vectorize(lambda th: T.attainable_bound(i, 32, 2.0**-53, u_mv, th))(theta)
        assert np.all(gap <= bound)


def test_thm4_bound_holds_for_preconditioned_run():
    wl = W.draw(20, 256, 32, 1, 16, 20.0, 0.8, 0.8, seed=22)
    A, b = D.gram(wl.H, wl.Y, wl.sigma2)
    L = 8
    C = np.zeros_like(A)
    for j in range(32 // L):
        sl = slice(j * L, (j + 1) * L)
        C[:, sl, sl] = np.linalg.cholesky(A[:, sl, sl])
    Ci = np.linalg.inv(C)
    Abar = Ci @ A @ np.conj(np.swapaxes(Ci, -1, -2))
    bbar = Ci @ b
    xs = np.linalg.solve(Abar, bbar)
    tr = []
    D.fp_cg(Abar, bbar, 15, D.paper_schedule(u_mv="fp16"), trace=tr)
    norms = [np.linalg.norm(x, axis=-2) for x, _ in tr]
    nx = np.linalg.norm(xs, axis=-2)
    for i, (x, r) in enumerate(tr, start=1):
        theta = np.max(np.stack(norms[:i]), axis=0) / nx
        gap = T.residual_gap(Abar, bbar, x, r, xs)
        bound = np.vectorize(lambda th: T.attainable_bound(i, 32, 2.0**-53, 2.0**-11, th))(theta)
        assert np.all(gap <= bound)


# ---------------------------------------------------------------- Thm 5 / Remark 5
def _kappa(a):
    w = np.linalg.eigvalsh(a)
    return w[-1] / w[0]


def _block_scaled(A, D_blocks, L):
    K = A.shape[0]
    C = np.zeros_like(A)
    for j in range(K // L):
        sl = slice(j * L, (j + 1) * L)
        C[sl, sl] = np.linalg.cholesky(D_blocks[j])
    Ci = np.linalg.inv(C)
    return Ci @ A @ Ci.conj().T


def test_remark5_bj_within_factor_d_of_any_block_scaling():
    rng = np.random.default_rng(5)
    K, L = 16, 4
    d = K // L
    for trial in range(20):
        wl = W.draw(1, 64, K, 1, 4, 15.0, 0.7, 0.7, seed=200 + trial)
        A, _ = D.gram(wl.H, wl.Y, wl.sigma2)
        A = A[0]
        kbj = _kappa(_block_scaled(A, [A[j * L:(j + 1) * L, j * L:(j + 1) * L] for j in range(d)], L))
        for _ in range(5):
            blocks = []
            for j in range(d):
                g = rng.standard_normal((L, L)) + 1j * rng.standard_normal((L, L))
                blocks.append(g @ g.conj().T + 0.5 * np.eye(L))
            assert kbj <= d * _kappa(_block_scaled(A, blocks, L)) * (1 + 1e-10)


def test_thm5_block_diagonal_gram_gives_identity():
    rng = np.random.default_rng(6)
    K, nue, L = 16, 4, 8
    blocks = []
    for _ in range(K // nue):
        h = rng.standard_normal((128, nue)) + 1j * rng.standard_normal((128, nue))
        blocks.append(h.conj().T @ h / 128 + 0.01 * np.eye(nue))
    A = sla.block_diag(*blocks)
    Abar = _block_scaled(A, [A[j * L:(j + 1) * L, j * L:(j + 1) * L] for j in range(K // L)], L)
    assert np.allclose(Abar, np.eye(K), atol=1e-12)
    assert _kappa(A) > 1.0 + 1e-6
