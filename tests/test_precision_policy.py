"""Host-side policies of the product: per-channel format selection from kappa
(eq. heuristic applied per channel) and the block-size choice by the
break-even rule of Remark 4."""
import numpy as np
import pytest

from paper_2504_09820_amd import precision as P


def test_formats_follow_the_heuristic_bound():
    K = 32
    # u < 1 / (K^1.5 sqrt(kappa)): fp16 (2^-11) needs kappa < (2^11 / K^1.5)^2
    k16 = (2.0**11 / K**1.5) ** 2
    f = P.formats_per_channel(np.array([1.0, 0.99 * k16, 1.01 * k16, np.nan, 0.5]), K)
    assert list(f) == ["fp16", "fp16", "fp32", "fp64", "fp64"]
    f = P.formats_per_channel(np.array([2.0]), K, allowed=("fp32",))
    assert list(f) == ["fp32"]


def test_cg_iteration_bound():
    assert P.cg_iterations(1.0) == 1
    # 2 ((10 - 1) / (10 + 1))^i < 1e-3  <=>  i > ln(2000) / ln(11 / 9) = 37.9
    assert P.cg_iterations(100.0) == 38
    ks = [P.cg_iterations(k) for k in (2.0, 10.0, 100.0, 1e4)]
    assert ks == sorted(ks)
    with pytest.raises(ValueError):
        P.cg_iterations(0.5)


def test_remark_five_cost_example():
    # K = 32, L = 8: the block-Jacobi setup costs as much as two iterations
    assert P.bj_setup_over_iteration(32, 8) == 2.0
    assert P.bj_setup_over_iteration(32, 0) == 0.0


def test_break_even_rule():
    K = 32
    k_plain = 60.0
    n0 = P.cg_iterations(k_plain)
    # find kappa values for L = 8 whose bound saves exactly 2 and exactly 3 iterations
    grid = np.linspace(1.0, k_plain, 20000)
    saves = {int(n0 - P.cg_iterations(k)): k for k in grid}
    L, tot = P.choose_block_size(K, {0: k_plain, 8: saves[2]})
    assert L == 0 and tot[0] == tot[8]            # saving = C_BJ / C^it: no gain, the smaller L
    L, _ = P.choose_block_size(K, {0: k_plain, 8: saves[3]})
    assert L == 8
    # larger blocks cost L^2 / K iterations: L = 16 needs a saving above 8
    L, _ = P.choose_block_size(K, {0: k_plain, 16: saves[8]})
    assert L == 0
