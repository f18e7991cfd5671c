"""Zero-forcing (sigma^2 = 0, A = H^H H) through the C ABI: FP64 against the
oracle and noise-free symbol recovery; the benchmarked fp16 symmetric
FP-BJ-CG schedule against the oracle's rounding-order spread."""
import sys

import numpy as np
import pytest

import workload as W
from tests.gpu_common import gpu_detect, oracle_detect, oracle_spread, quantiles

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("L,variant", [(0, 0), (4, 2), (8, 0)])
def test_zero_forcing_fp64_recovers_noise_free_symbols(L, variant):
    wl = W.draw(12, 64, 16, 5, 64, 30.0, 0.5, 0.5, seed=21)
    wl.sigma2[:] = 0.0
    Y = wl.H @ wl.X
    _say(f"case ZF fp64 L={L} v{variant}")
    # I = 2K: converged (finite precision loses the K-step termination; the
    # residual reaches 1e-19 of its start by about 21 steps here)
    x, lab, fl = gpu_detect(wl, 64, 32, L, "fp64", variant=variant, Y=Y)
    ref = oracle_detect(wl, 64, 32, L, "fp64", variant=variant, Y=Y)
    rel = np.linalg.norm(x - ref.xhat, axis=-2) / np.linalg.norm(ref.xhat, axis=-2)
    assert rel.max() < 1e-12, rel.max()
    np.testing.assert_allclose(x, wl.X, atol=1e-9)
    assert np.array_equal(lab, wl.labels) and np.all(fl == 0)


def test_zero_forcing_fp16_symmetric_matches_oracle_spread():
    wl = W.draw(8, 128, 32, 14, 64, 25.0, 0.5, 0.5, seed=22)
    wl.sigma2[:] = 0.0                                 # noisy Y, zero-forcing system
    _say("case ZF fp16 L=4 symmetric, I=11")
    x, lab, fl = gpu_detect(wl, 64, 11, 4, "fp16", io=np.complex64, variant=2)
    spread, ref = oracle_spread(wl, 64, 11, 4, "fp16", np.complex64, variant=2)
    ref_x = ref.xhat.astype(np.complex64).astype(np.complex128)
    nrm = np.linalg.norm(ref.xhat, axis=-2)
    qg = quantiles(np.linalg.norm(x - ref_x, axis=-2) / nrm)
    qs = quantiles(spread / nrm)
    _say(f"  gpu-oracle {qg}  oracle spread {qs}")
    assert np.all(qg <= 4.0 * qs + 18 * 2.0**-24), (qg, qs)
    assert np.all(fl == ref.flags)
