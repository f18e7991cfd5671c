"""Detection on the robustness workloads (Sec. V: imperfect CSI, geometry-based
multipath, Gauss-Markov time variation) through the C ABI: FP64 converged
against the oracle, the timed fp16 symmetric FP-BJ-CG schedule within the
oracle's rounding-order spread."""
import sys

import numpy as np
import pytest

import workload as W
from tests.gpu_common import gpu_detect, oracle_detect, oracle_spread, quantiles

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _workloads():
    base = W.draw(8, 128, 32, 14, 64, 22.0, 0.5, 0.5, seed=61)
    gm = W.gauss_markov(8, 128, 32, 14, 64, 22.0, 0.5, 0.5, 3, 1000.0, seed=62)
    return {"csi20": W.imperfect_csi(base, 20.0, seed=63), "csi25": W.imperfect_csi(base, 25.0, seed=64),
            "geometry": W.geometry(8, 128, 32, 14, 64, 22.0, seed=65), "gm-step2": gm[2]}


@pytest.mark.parametrize("name", ["csi20", "csi25", "geometry", "gm-step2"])
def test_robust_workloads_match_oracle(name):
    wl = _workloads()[name]
    _say(f"case robustness workload {name}")
    x, lab, fl = gpu_detect(wl, 64, 96, 4, "fp64", variant=2)             # converged FP64
    ref = oracle_detect(wl, 64, 96, 4, "fp64", variant=2)
    rel = np.linalg.norm(x - ref.xhat, axis=-2) / np.linalg.norm(ref.xhat, axis=-2)
    assert rel.max() < 1e-12, rel.max()
    x, lab, fl = gpu_detect(wl, 64, 11, 4, "fp16", io=np.complex64, variant=2)
    spread, ref = oracle_spread(wl, 64, 11, 4, "fp16", np.complex64, variant=2)
    ref_x = ref.xhat.astype(np.complex64).astype(np.complex128)
    nrm = np.linalg.norm(ref.xhat, axis=-2)
    qg = quantiles(np.linalg.norm(x - ref_x, axis=-2) / nrm)
    qs = quantiles(spread / nrm)
    _say(f"  fp16 gpu-oracle {qg}  oracle spread {qs}")
    assert np.all(qg <= 4.0 * qs + 18 * 2.0**-24), (qg, qs)
    assert np.all(fl == ref.flags)
