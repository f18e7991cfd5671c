"""The benchmark's algorithmic byte and flop counts, on which its roofline
figures rest, against counts written out by hand for the workloads it
reports (CPU only)."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_algorithmic_bytes_c3(bench):
    # per channel: H 256 x 64 and Y 256 x 14 complex64 in, sigma^2 (8 B) in,
    # x_hat 64 x 14 complex64, labels 64 x 14 bytes and a 4-byte flag word out
    per = 256 * 64 * 8 + 256 * 14 * 8 + 8 + 64 * 14 * 8 + 64 * 14 + 4
    assert per == 167820
    assert bench.algorithmic_bytes(8192, 256, 64, 14) == 8192 * per
    # complex128 inputs double the element bytes; a refinement step reads H, Y again
    per128 = 256 * 78 * 16 + 8 + 64 * 14 * 16 + 64 * 14 + 4
    assert bench.algorithmic_bytes(1, 256, 64, 14, elem=16) == per128
    assert bench.algorithmic_bytes(1, 256, 64, 14, refine=1) == per + 256 * 78 * 8


def test_work_model_counts(bench):
    B, Nbs, K, R, L, I = 8192, 256, 64, 14, 4, 20
    w = bench.work_model(B, Nbs, K, R, L, I, "fp16", refresh=4)
    gram = 4 * K * (K + 1) * Nbs + 8 * K * Nbs * R
    cg = I * R * (8 * K * K + 40 * K + 8 * K * L) + 8 * K * L * L
    assert w["lowp_flops"] == pytest.approx(B * (gram + cg))
    # refreshes at iterations 4, 8, 12, 16 (not after the last one)
    assert w["fp64_flops"] == pytest.approx(B * 4 * R * 8 * K * K)
    # the FP64 schedule counts everything as FP64 work
    w64 = bench.work_model(B, Nbs, K, R, 0, 27, "fp64")
    assert w64["lowp_flops"] == 0
    assert w64["fp64_flops"] == pytest.approx(B * (gram + 27 * R * (8 * K * K + 40 * K)))
    # refinement: one more solve and the FP64 residual through H per step
    wr = bench.work_model(2048, 512, 128, 14, 16, 16, "fp8", refine=1)
    g4 = 4 * 128 * 129 * 512 + 8 * 128 * 512 * 14
    cg4 = 16 * 14 * (8 * 128 * 128 + 40 * 128 + 8 * 128 * 16) + 8 * 128 * 16 * 16
    assert wr["lowp_flops"] == pytest.approx(2048 * (g4 + 2 * cg4))
    assert wr["fp64_flops"] == pytest.approx(2048 * 16 * 512 * 128 * 14)


def test_roofline_picks_the_binding_roof(bench):
    # c3's configured schedule: the FP64 refreshes take longer at peak than
    # the HBM stream and the fp16 products, so they bind
    w = bench.work_model(8192, 256, 64, 14, 4, 20, "fp16", refresh=4)
    r = bench.roofline_of(w, "fp16", 0.6)
    t = {k: v["time_at_peak_us"] for k, v in r["roofs"].items()}
    assert r["roof"] == max(t, key=t.get) == "mfma_fp64"
    assert r["frac"] == pytest.approx(w["fp64_flops"] / 0.6e-3 / 78.6e12, rel=1e-3)
    assert r["roofs"]["hbm"]["time_at_peak_us"] == pytest.approx(8192 * 167820 / 8e12 * 1e6, abs=0.01)
    # without the refresh the same launch is bound by HBM
    w0 = bench.work_model(8192, 256, 64, 14, 4, 20, "fp16")
    assert bench.roofline_of(w0, "fp16", 0.6)["roof"] == "hbm"
