"""C-ABI contract checks that need no GPU: the library loads, exports every
function declared in include/fpcg.h, validates arguments on the host exactly
as documented, and its precision heuristic agrees with the oracle's."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="session")
def fp():
    import paper_2504_09820_amd as fp

    if not os.path.exists(fp.library_path):
        from paper_2504_09820_amd import build

        build.build(incremental=True, verbose=False)
    fp.lib()
    return fp


def _declared():
    txt = open(os.path.join(ROOT, "include", "fpcg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fpcg_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(fp):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(fp.lib(), n), n


def test_strerror_codes(fp):
    L = fp.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.fpcg_strerror(code).decode()
    assert L.fpcg_strerror(-99).decode() == "unknown status"


def test_check_accepts_built_configurations(fp):
    for name in ("fp64", "fp32", "bf16", "fp16", "fp8"):
        s = fp.schedule(name)
        assert fp.check(1000, 64, 8, 1, 16, 8, 0, s) == 0 or name == "fp8"
        assert fp.check(16384, 128, 32, 14, 64, 16, 0, s) == 0
        assert fp.check(8192, 256, 64, 14, 64, 16, 8, s) == 0
        assert fp.check(10, 256, 64, 14, 64, 16, 4, fp.schedule(name, refresh_every=4)) == 0
    assert fp.check(0, 1, 1, 1, 4, 0, 0, None) == 0          # empty batch, FP64 default
    assert fp.check(3, 1, 1, 1, 4, 1, 0, fp.schedule("fp64")) == 0
    assert fp.check(3, 50, 20, 17, 16, 5, 4, fp.schedule("fp32", refine_steps=2)) == 0
    assert fp.check(1, 2**20 - 1, 128, 1, 16, 8, 0, fp.schedule("fp16")) == 0   # just below 2 GiB


@pytest.mark.parametrize("args,code", [
    ((-1, 64, 8, 1, 16, 8, 0), -1),
    ((2**31, 64, 8, 1, 16, 8, 0), -1),
    ((10, 0, 8, 1, 16, 8, 0), -1),
    ((10, 64, 0, 1, 16, 8, 0), -1),
    ((10, 64, 8, 0, 16, 8, 0), -1),
    ((10, 64, 8, 1, 8, 8, 0), -1),      # not a square QAM order
    ((10, 64, 8, 1, 16, -1, 0), -1),
    ((10, 64, 8, 1, 16, 8, 3), -1),     # L does not divide K
    ((10, 64, 8, 1, 16, 8, -4), -1),
    ((10, 256, 128, 1, 16, 8, 8), -4),  # K = 128 with fp32 operands: no preconditioner only
    ((10, 512, 192, 1, 16, 8, 0), -4),  # K > 128 not built
    ((10, 64, 32, 1, 16, 8, 16), -4),   # L = 16 not built for fp32 operands
    ((10, 64, 32, 1, 16, 8, 32), -4),   # L = 32 not built
    ((10, 64, 16, 1, 16, 8, 2), -4),    # L = 2 not built
    ((10, 2**24, 8, 1, 16, 8, 0), -4),     # one channel's H reaches 2 GiB (complex128)
    ((10, 64, 8, 2**21, 16, 8, 0), -4),    # one channel's Y reaches 2 GiB
])
def test_check_rejects(fp, args, code):
    assert fp.check(*args, fp.schedule("fp32")) == code


def test_check_large_k(fp):
    s8 = fp.schedule("fp8", refine_steps=1)
    assert fp.check(2048, 512, 128, 14, 256, 16, 16, s8) == 0
    assert fp.check(5, 512, 100, 14, 256, 16, 0, fp.schedule("fp8")) == 0
    assert fp.check(5, 512, 112, 14, 256, 16, 16, fp.schedule("fp8")) == 0
    assert fp.check(5, 512, 120, 14, 256, 16, 8, fp.schedule("fp8")) == 0
    assert fp.check(5, 512, 128, 14, 256, 16, 16, fp.schedule("fp16")) == 0
    assert fp.check(5, 512, 128, 14, 256, 16, 0, fp.schedule("bf16")) == 0
    assert fp.check(5, 512, 128, 14, 256, 16, 16, fp.schedule("fp8", variant=2)) == -4      # symmetric form
    assert fp.check(5, 512, 128, 14, 256, 16, 16, fp.schedule("fp8", refresh_every=4)) == -4   # refresh
    assert fp.check(5, 512, 128, 14, 256, 16, 16, fp.schedule("fp16", refine_steps=1)) == -4   # LDS
    assert fp.check(5, 512, 128, 14, 256, 16, 16, fp.schedule("fp64")) == -4
    assert fp.check(2048, 512, 128, 14, 256, 48, 0, fp.schedule("fp64")) == 0      # slab form
    assert fp.check(2048, 512, 128, 14, 256, 48, 0, fp.schedule("fp32")) == 0
    assert fp.check(5, 512, 128, 14, 256, 16, 0, fp.schedule("fp32", refresh_every=4)) == -4
    assert fp.check(5, 512, 128, 14, 256, 16, 0, fp.schedule("fp64", refine_steps=1)) == -4
    assert fp.check(5, 256, 64, 14, 64, 16, 4, fp.schedule("fp16", refresh_every=4, variant=2)) == 0
    assert fp.check(5, 256, 32, 14, 64, 16, 16, fp.schedule("fp16")) == 0      # L = 16 runs the K <= 128 build


def test_check_slab_block_sizes(fp):
    """The slab form's block-Jacobi builds: L = 8 (K <= 64) and L = 16 in the
    symmetric form only, with or without the FP64 refresh; L = 16 at
    K = 128 for fp32, fp16 and bf16 but not fp8 or FP64."""
    sch = fp.schedule
    assert fp.check(5, 256, 64, 14, 64, 16, 8, sch("fp16", refresh_every=4, variant=2)) == 0
    assert fp.check(5, 256, 56, 14, 64, 16, 8, sch("fp32", variant=2)) == 0
    assert fp.check(5, 256, 64, 14, 64, 16, 16, sch("fp32", variant=2)) == 0
    assert fp.check(5, 256, 64, 14, 64, 16, 16, sch("fp32", refresh_every=3, variant=2)) == 0
    for f in ("fp32", "fp16", "bf16"):
        assert fp.check(5, 512, 128, 14, 256, 16, 16, sch(f, variant=2)) == 0
        assert fp.check(5, 512, 128, 14, 256, 16, 16, sch(f, refresh_every=4, variant=2)) == 0
        assert fp.check(5, 512, 112, 14, 256, 16, 16, sch(f, variant=2)) == 0
    assert fp.check(5, 512, 128, 14, 256, 16, 16, sch("fp32", variant=0)) == -4     # no left form there
    assert fp.check(5, 512, 128, 14, 256, 16, 16, sch("fp16", refresh_every=4, variant=0)) == -4
    assert fp.check(5, 512, 128, 14, 256, 16, 16, sch("fp64", variant=2)) == -4
    assert fp.check(5, 512, 128, 14, 256, 16, 8, sch("fp32", variant=2)) == -4


def test_check_rejects_bad_schedules(fp):
    S = fp.Schedule
    assert fp.check(4, 64, 8, 1, 16, 8, 0, S(9, 9, 1, 1, 0, 0, 0)) == -1
    assert fp.check(4, 64, 8, 1, 16, 8, 0, S(1, 1, 1, 1, -1, 0, 0)) == -1
    assert fp.check(4, 64, 8, 1, 16, 8, 0, S(1, 1, 1, 1, 0, 99, 0)) == -1
    assert fp.check(4, 64, 8, 1, 16, 8, 0, S(1, 1, 1, 1, 0, 0, 3)) == -1
    assert fp.check(4, 64, 8, 1, 16, 8, 4, S(1, 1, 1, 1, 0, 0, 2)) == 0
    assert fp.check(4, 64, 8, 1, 16, 8, 0, S(1, 2, 1, 1, 0, 0, 0)) == -4   # gram_op != mv_op
    assert fp.check(4, 64, 8, 1, 16, 8, 0, S(2, 2, 0, 0, 0, 0, 0)) == -4   # FP64 work with bf16 operands
    assert fp.check(4, 64, 8, 1, 16, 8, 0, S(0, 0, 1, 1, 0, 0, 0)) == -4   # FP32 work with FP64 operands


def test_last_error_message(fp):
    assert fp.check(10, 64, 8, 1, 16, 8, 3, fp.schedule("fp32")) == -1
    assert "divide" in fp.lib().fpcg_last_error().decode()


def test_select_precision_matches_oracle_heuristic(fp):
    from oracle import theory as T

    for N in (8, 16, 32, 64, 100, 128):
        for kappa in (1.0, 2.0, 5.0, 17.25, 50.0, 245.0, 1e3, 1e5, 1e9):
            for allow in (True, False):
                name, u = fp.select_precision(N, kappa, allow)
                ref = T.select_format(N, kappa, allow_fp8=allow)
                assert {"fp8": "e4m3"}.get(name, name) == ref, (N, kappa, allow)
                assert u == pytest.approx(T.heuristic_bound(N, kappa), rel=1e-14)


def test_select_precision_rejects(fp):
    f = ctypes.c_int32()
    assert fp.lib().fpcg_select_precision(0, 10.0, 1, ctypes.byref(f), None) == -1
    assert fp.lib().fpcg_select_precision(8, 0.5, 1, ctypes.byref(f), None) == -1
    assert fp.lib().fpcg_select_precision(8, float("nan"), 1, ctypes.byref(f), None) == -1


def test_no_cpu_fallback_without_device(fp):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(fp.FpcgError):
        fp.Context(0)


def test_launch_form_rejects_unknown(fp):
    L = fp.lib()
    assert L.fpcg_set_launch_form(None, 0) == -1


def test_autotune_validates_before_touching_a_device(fp):
    L = fp.lib()
    s = fp.schedule("fp16")
    import ctypes as ct

    out = ct.c_int32(-7)
    assert L.fpcg_autotune(None, None, 16, 128, 32, 14, 1, 64, 8, 4, ct.byref(s), 3, ct.byref(out)) == -1
    assert out.value == -7


def test_demap_validates_on_the_host(fp):
    L = fp.lib()
    buf = ctypes.create_string_buffer(64)
    p = ctypes.addressof(buf)
    al = (p + 15) & ~15
    assert L.fpcg_demap_maxlog(None, 0, 1, None, 1, None, 64, None) == 0          # empty: nothing to do
    assert L.fpcg_demap_maxlog(None, -1, 1, p, 1, p, 64, al) == -1
    assert L.fpcg_demap_maxlog(None, 4, 0, p, 1, p, 64, al) == -1                 # R < 1
    for q in (2, 8, 32, 1024):
        assert L.fpcg_demap_maxlog(None, 4, 1, p, 1, p, q, al) == -1
    assert L.fpcg_demap_maxlog(None, 4, 1, None, 1, p, 16, al) == -1
    assert L.fpcg_demap_maxlog(None, 4, 1, p, 1, None, 16, al) == -1
    assert L.fpcg_demap_maxlog(None, 4, 1, p, 1, p, 16, None) == -1
    assert L.fpcg_demap_maxlog(None, 4, 1, p, 1, p, 16, al + 4) == -1             # llr not 16-byte aligned
    assert "aligned" in L.fpcg_last_error().decode()
    i8 = L.fpcg_demap_maxlog_i8
    assert i8(None, 0, 1, None, 1, None, 64, 4.0, None) == 0
    for sc in (0.0, -1.0, float("inf"), float("nan")):
        assert i8(None, 4, 1, p, 1, p, 16, sc, al) == -1
    assert i8(None, 4, 1, p, 1, p, 16, 4.0, al + 4) == -1                         # int8 LLRs 8-byte aligned
    assert i8(None, 4, 0, p, 1, p, 16, 4.0, al) == -1


def _bare_server(fp, chans=None):
    """A Server object with a NULL library handle: the binding's own checks run,
    and anything that reaches the library is refused there (NULL server)."""
    srv = fp.Server.__new__(fp.Server)
    srv._h = ctypes.c_void_p()
    srv._keep = {}
    srv._chans = dict(chans or {})
    return srv


def test_server_submit_validates_shapes_before_the_library(fp):
    import numpy as np

    srv = _bare_server(fp, {7: (4, 16, 8, np.complex64)})
    H = np.zeros((4, 16, 8), np.complex64)
    Y = np.zeros((4, 16, 3), np.complex64)
    s2 = np.ones(4)
    bad = [
        dict(H=H, Y=np.zeros((3, 16, 3), np.complex64), sigma2=s2),     # B of Y differs
        dict(H=H, Y=np.zeros((4, 15, 3), np.complex64), sigma2=s2),     # Nbs of Y differs
        dict(H=H, Y=np.zeros((4, 16), np.complex64), sigma2=s2),        # Y not 3-D
        dict(H=H, Y=Y, sigma2=np.ones(3)),                              # sigma2 too short
        dict(H=H, Y=Y, sigma2=np.ones((4, 1))),                         # sigma2 not (B,)
        dict(H=np.zeros((4, 16, 8), np.float32), Y=Y, sigma2=s2),       # H not complex
        dict(H=None, Y=np.zeros((4, 17, 3), np.complex64), sigma2=None, channels=7),   # resident set: Nbs
        dict(H=None, Y=np.zeros((2, 16, 3), np.complex64), sigma2=None, channels=7),   # resident set: B
        dict(H=None, Y=Y, sigma2=None, channels=8),                                    # unknown handle
    ]
    for kw in bad:
        with pytest.raises((ValueError, TypeError)):
            srv.submit(qam=16, iters=4, **kw)
    # consistent shapes reach the library, which refuses the NULL server
    with pytest.raises(fp.FpcgError):
        srv.submit(H, Y, s2, 16, 4)
    with pytest.raises(fp.FpcgError):
        srv.submit(None, Y, None, 16, 4, channels=7)


def test_tune_table_is_validated_before_any_device_call(fp):
    L = fp.lib()
    h = ctypes.c_void_p()
    for bad in (b"", b"[]", b"{", b'{"forms": [{"KP": 64}]}', b'{"kappa": [{"Nbs": 1, "K": 2, "L": 0, "kappa": 0.5}]}',
                b'{"forms": [{"KP": 64, "fmt": 3, "L": 4, "split": 1, "refresh": 1, "c64": 1, "multi": 0, "form": 7}]}',
                b'{"forms": []} x'):
        assert L.fpcg_create(0, 0, bad, ctypes.byref(h)) == -1, bad
        assert "tune table" in L.fpcg_last_error().decode()
    good = (b'{"version": 1, "note": "x", "forms": [{"KP": 64, "fmt": 3, "L": 4, "split": 1, "refresh": 1, "c64": 1, '
            b'"multi": 0, "form": 1025}], "kappa": [{"Nbs": 256, "K": 64, "L": 4, "kappa": 37.9}]}')
    import torch

    st = L.fpcg_create(0, 0, good, ctypes.byref(h))
    if torch.cuda.is_available():
        assert st == 0
        L.fpcg_destroy(h)
    else:
        assert st == -3                    # parsed, then no device


def test_policy_calls_validate_on_the_host(fp):
    L = fp.lib()
    n = ctypes.c_size_t()
    assert L.fpcg_tune_table(None, None, 0, ctypes.byref(n)) == -1
    assert L.fpcg_set_kappa(None, 256, 64, 4, 10.0) == -1
    k = ctypes.c_double()
    assert L.fpcg_expected_kappa(None, None, 8, 256, 64, 14, None, None, 1, None, 4, 16, ctypes.byref(k)) == -1
    s = fp.schedule("fp8")
    assert L.fpcg_gram(None, None, 8, 64, 32, 14, None, None, 1, None, ctypes.byref(s), None, None, None) == -1


def test_detect_pc_rejects_mode_and_block_size_before_anything_else():
    """fpcg_detect_pc: the mode and block size are checked first (no context
    or device needed), with FPCG_E_INVAL and a message."""
    import ctypes

    import paper_2504_09820_amd as fp

    L = fp.lib()
    args = [None, None, 4, 64, 16, 2, None, None, 1, None, 16, 4]
    st = L.fpcg_detect_pc(*args, 4, None, None, None, None, None, 3)
    assert st == fp.E_INVAL and b"mode" in L.fpcg_last_error()
    st = L.fpcg_detect_pc(*args, 0, None, None, None, None, None, fp.PRECOND_STORE)
    assert st == fp.E_INVAL and b"block_L" in L.fpcg_last_error()
    st = L.fpcg_detect_pc(*args, 4, None, None, None, None, None, fp.PRECOND_LOAD)
    assert st == fp.E_INVAL and b"ctx" in L.fpcg_last_error()
