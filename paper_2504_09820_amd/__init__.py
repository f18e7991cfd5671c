"""MI355X (gfx950) finite-precision block-Jacobi CG massive-MIMO detector.

A thin ctypes binding of the C ABI in include/fpcg.h (libfpcg.so, built by
``paper_2504_09820_amd.build``).  It only marshals arguments: every step of
the detector runs in the library's HIP kernels.  PyTorch is used for device
memory and streams.  If the library is missing the calls raise; there is no
CPU fallback.

    ctx = Context()
    xhat, labels, flags = detect(H, Y, sigma2, qam=64, iters=16, schedule="bf16")
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

__all__ = [
    "FMT", "FLAGS", "Schedule", "schedule", "Context", "FpcgError", "lib", "library_path",
    "detect", "check", "gram", "slice_qam", "demap_maxlog", "round_operand", "select_precision", "Server",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libfpcg.so")

FMT = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3, "fp8": 4, "e4m3": 4}
FMT_NAME = {0: "fp64", 1: "fp32", 2: "bf16", 3: "fp16", 4: "fp8"}
FLAGS = {"nonfinite": 1, "breakdown": 2, "block_not_pd": 4, "fp8_sat": 8}

OK, E_INVAL, E_NOMEM, E_DEVICE, E_UNSUPPORTED, E_BUSY = 0, -1, -2, -3, -4, -5
PRECOND_STORE, PRECOND_LOAD = 1, 2


class FpcgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fpcg status {status}: {msg}")
        self.status = status


class Schedule(ctypes.Structure):
    _fields_ = [
        ("gram_op", ctypes.c_int32), ("mv_op", ctypes.c_int32), ("ip", ctypes.c_int32), ("work", ctypes.c_int32),
        ("refresh_every", ctypes.c_int32), ("refine_steps", ctypes.c_int32), ("variant", ctypes.c_int32),
    ]


def schedule(name: str = "fp64", refresh_every: int = 0, refine_steps: int = 0, variant: int = 0) -> Schedule:
    """Named schedule: operands of the Gram and of A p in ``name``; u_IP = u_W =
    FP64 for "fp64", FP32 otherwise."""
    f = FMT[name]
    w = 0 if f == 0 else 1
    return Schedule(f, f, w, w, refresh_every, refine_steps, variant)


class _Request(ctypes.Structure):
    _fields_ = [
        ("B", ctypes.c_int64), ("Nbs", ctypes.c_int32), ("K", ctypes.c_int32), ("R", ctypes.c_int32),
        ("io_c64", ctypes.c_int32), ("qam_order", ctypes.c_int32), ("iters", ctypes.c_int32),
        ("block_L", ctypes.c_int32), ("sched", Schedule),
        ("H", ctypes.c_void_p), ("Y", ctypes.c_void_p), ("sigma2", ctypes.c_void_p),
        ("xhat", ctypes.c_void_p), ("labels", ctypes.c_void_p), ("flags", ctypes.c_void_p),
        ("channels", ctypes.c_uint64),
    ]


_lib = None


def lib():
    """Load libfpcg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(library_path):
        raise FpcgError(E_DEVICE, f"{library_path} is not built; run `python -m paper_2504_09820_amd.build`")
    # torch first: the library's HIP runtime dependency then binds to the runtime
    # torch has loaded (same soname), so the process holds one HIP runtime and
    # torch's device memory and streams are that runtime's own
    import torch  # noqa: F401

    L = ctypes.CDLL(library_path)
    st = ctypes.c_int32
    vp = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    L.fpcg_create.argtypes = [i32, ctypes.c_size_t, ctypes.c_char_p, ctypes.POINTER(vp)]
    L.fpcg_create.restype = st
    L.fpcg_tune_table.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    L.fpcg_tune_table.restype = st
    L.fpcg_set_kappa.argtypes = [vp, i32, i32, i32, ctypes.c_double]
    L.fpcg_set_kappa.restype = st
    L.fpcg_expected_kappa.argtypes = [vp, vp, i64, i32, i32, i32, vp, vp, i32, vp, i32, i32,
                                      ctypes.POINTER(ctypes.c_double)]
    L.fpcg_expected_kappa.restype = st
    L.fpcg_destroy.argtypes = [vp]
    L.fpcg_destroy.restype = None
    L.fpcg_set_launch_form.argtypes = [vp, i32]
    L.fpcg_set_launch_form.restype = st
    L.fpcg_autotune.argtypes = [vp, vp, i64, i32, i32, i32, i32, i32, i32, i32, ctypes.POINTER(Schedule), i32,
                                ctypes.POINTER(i32)]
    L.fpcg_autotune.restype = st
    L.fpcg_server_channels.argtypes = [vp, i64, i32, i32, i32, vp, vp, ctypes.POINTER(ctypes.c_uint64)]
    L.fpcg_server_channels.restype = st
    L.fpcg_server_release.argtypes = [vp, ctypes.c_uint64]
    L.fpcg_server_release.restype = st
    L.fpcg_server_channels_update.argtypes = [vp, ctypes.c_uint64, vp, vp, i32]
    L.fpcg_server_channels_update.restype = st
    L.fpcg_strerror.argtypes = [i32]
    L.fpcg_strerror.restype = ctypes.c_char_p
    L.fpcg_last_error.argtypes = []
    L.fpcg_last_error.restype = ctypes.c_char_p
    L.fpcg_check.argtypes = [i64, i32, i32, i32, i32, i32, i32, ctypes.POINTER(Schedule)]
    L.fpcg_check.restype = st
    L.fpcg_detect.argtypes = [vp, vp, i64, i32, i32, i32, vp, vp, i32, vp, i32, i32, i32, ctypes.POINTER(Schedule), vp, vp, vp]
    L.fpcg_detect.restype = st
    L.fpcg_detect_ex.argtypes = [vp, vp, i64, i32, i32, i32, vp, vp, i32, vp, i32, i32, i32, ctypes.POINTER(Schedule),
                                 vp, vp, vp, vp, i64, vp, vp]
    L.fpcg_detect_ex.restype = st
    L.fpcg_detect_ex_static.argtypes = L.fpcg_detect_ex.argtypes
    L.fpcg_detect_ex_static.restype = st
    L.fpcg_detect_pc.argtypes = L.fpcg_detect.argtypes + [vp, i32]
    L.fpcg_detect_pc.restype = st
    L.fpcg_gram.argtypes = [vp, vp, i64, i32, i32, i32, vp, vp, i32, vp, ctypes.POINTER(Schedule), vp, vp, vp]
    L.fpcg_gram.restype = st
    L.fpcg_demap_maxlog.argtypes = [vp, i64, i32, vp, i32, vp, i32, vp]
    L.fpcg_demap_maxlog.restype = st
    L.fpcg_demap_maxlog_i8.argtypes = [vp, i64, i32, vp, i32, vp, i32, ctypes.c_float, vp]
    L.fpcg_demap_maxlog_i8.restype = st
    L.fpcg_slice.argtypes = [vp, i64, vp, i32, i32, vp]
    L.fpcg_slice.restype = st
    L.fpcg_round.argtypes = [vp, i64, vp, i32, ctypes.c_float, vp]
    L.fpcg_round.restype = st
    L.fpcg_select_precision.argtypes = [i32, ctypes.c_double, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    L.fpcg_select_precision.restype = st
    L.fpcg_server_create.argtypes = [vp, i32, i32, ctypes.POINTER(vp)]
    L.fpcg_server_create.restype = st
    L.fpcg_submit.argtypes = [vp, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)]
    L.fpcg_submit.restype = st
    L.fpcg_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32)]
    L.fpcg_poll.restype = st
    L.fpcg_drain.argtypes = [vp]
    L.fpcg_drain.restype = st
    L.fpcg_server_stats.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_size_t)]
    L.fpcg_server_stats.restype = st
    L.fpcg_server_destroy.argtypes = [vp]
    L.fpcg_server_destroy.restype = None
    _lib = L
    return L


def _check(status: int):
    if status != OK:
        raise FpcgError(status, lib().fpcg_last_error().decode() or lib().fpcg_strerror(status).decode())


def check(B, Nbs, K, R, qam, iters, L=0, sched: Optional[Schedule] = None) -> int:
    """Host-only validation; returns the status code (0 = accepted)."""
    return lib().fpcg_check(B, Nbs, K, R, qam, iters, L, ctypes.byref(sched) if sched is not None else None)


def select_precision(N: int, kappa: float, allow_fp8: bool = True):
    """eq. heuristic: returns (format name, u bound)."""
    f = ctypes.c_int32()
    u = ctypes.c_double()
    _check(lib().fpcg_select_precision(N, kappa, 1 if allow_fp8 else 0, ctypes.byref(f), ctypes.byref(u)))
    return FMT_NAME[f.value], u.value


LAUNCH_WAVES_SHIFT = 8


def _form_code(form: str) -> int:
    base = {"auto": 0, "fused": 1, "pipelined": 2, "slab": 3}
    if form in base:
        return base[form]
    if form.startswith("fused-w") and form[7:] in ("1", "2", "4"):
        return 1 | (int(form[7:]) << LAUNCH_WAVES_SHIFT)
    raise ValueError(f"unknown launch form {form!r}")


def _form_name(code: int) -> str:
    nw = code >> LAUNCH_WAVES_SHIFT
    base = {0: "auto", 1: "fused", 2: "pipelined", 3: "slab"}[code & ((1 << LAUNCH_WAVES_SHIFT) - 1)]
    return f"{base}-w{nw}" if nw else base


class Context:
    """A device context (fpcg_create / fpcg_destroy)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, tune_table: "str | dict | None" = None):
        """tune_table: a table from tune_table() (JSON text or its parsed dict)
        with launch forms and expected condition numbers to start from."""
        import json

        self._h = ctypes.c_void_p()
        tt = None
        if tune_table is not None:
            tt = (json.dumps(tune_table) if isinstance(tune_table, dict) else str(tune_table)).encode()
        _check(lib().fpcg_create(device, hbm_budget, tt, ctypes.byref(self._h)))
        self.device = device

    def tune_table(self) -> str:
        """The context's launch forms and expected condition numbers as JSON
        (fpcg_tune_table), to persist and pass to a later Context."""
        n = ctypes.c_size_t()
        _check(lib().fpcg_tune_table(self._h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().fpcg_tune_table(self._h, buf, n.value, ctypes.byref(n)))
        return buf.value.decode()

    def set_kappa(self, Nbs: int, K: int, L: int, kappa: float):
        """Record E{kappa} of the workload class (Nbs, K, L) for the heuristic
        schedule (detect with schedule_=None)."""
        _check(lib().fpcg_set_kappa(self._h, Nbs, K, L, float(kappa)))

    def expected_kappa(self, H, Y, sigma2, L: int = 0, sample: int = 64, stream=None) -> float:
        """E{kappa} of the iteration matrix estimated on the device from
        `sample` channels of the batch (fpcg_expected_kappa); also recorded in
        the context for the heuristic schedule."""
        import torch

        if not (H.is_cuda and Y.is_cuda and sigma2.is_cuda) or H.dtype != Y.dtype or \
                H.dtype not in (torch.complex64, torch.complex128) or sigma2.dtype != torch.float64:
            raise TypeError("H, Y: complex64/complex128 CUDA tensors of one dtype; sigma2: float64 CUDA tensor")
        H, Y, sigma2 = H.contiguous(), Y.contiguous(), sigma2.contiguous()
        B, Nbs, K = H.shape
        if Y.dim() != 3 or Y.shape[:2] != (B, Nbs) or sigma2.shape != (B,):
            raise ValueError("shape mismatch between H, Y and sigma2")
        out = ctypes.c_double()
        _check(lib().fpcg_expected_kappa(self._h, _stream_handle(stream, H.device), B, Nbs, K, Y.shape[2],
                                         ctypes.c_void_p(H.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                         1 if H.dtype == torch.complex64 else 0, ctypes.c_void_p(sigma2.data_ptr()),
                                         L, sample, ctypes.byref(out)))
        return out.value

    @property
    def handle(self):
        return self._h

    def autotune(self, B, Nbs, K, R, qam, iters, L=0, schedule_: "str | Schedule" = "fp64", refresh_every=0,
                 refine_steps=0, variant=0, io="complex64", reps=5, stream=None):
        """Time the launch forms built for this shape class and keep the fastest
        for launches in the "auto" form; returns its name."""
        import torch

        sched = schedule(schedule_, refresh_every, refine_steps, variant) if isinstance(schedule_, str) else schedule_
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        out = ctypes.c_int32()
        _check(lib().fpcg_autotune(self._h, ctypes.c_void_p(s.cuda_stream), B, Nbs, K, R, 1 if io == "complex64" else 0,
                                   qam, iters, L, ctypes.byref(sched), reps, ctypes.byref(out)))
        return _form_name(out.value)

    def set_launch_form(self, form: str = "auto"):
        """"auto" (the library's choice), "fused" (one workgroup per channel),
        "fused-w1" / "fused-w2" / "fused-w4" (the fused form with that many
        waves per channel where built for a launch's shape), "pipelined"
        (two-wave pipelined form where built) or "slab" (A held in registers
        across K/16 waves, K = 64 and 128)."""
        _check(lib().fpcg_set_launch_form(self._h, _form_code(form)))

    def close(self):
        if self._h:
            lib().fpcg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def _ctx_for(device: int) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def _stream_handle(stream, device):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _check_tensor(t, name, shape, dtype, device):
    """Caller-supplied arrays are written or read by the kernels at the sizes
    the call implies: reject anything else before a launch."""
    if not getattr(t, "is_cuda", False) or t.device != device:
        raise TypeError(f"{name} must be a CUDA tensor on {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def detect(H, Y, sigma2, qam: int, iters: int, L: int = 0, schedule_: "str | Schedule" = "fp64",
           refresh_every: int = 0, refine_steps: int = 0, variant: int = 0,
           ctx: Optional[Context] = None, stream=None, out=None, chan_idx=None, kappa=None, gain=None,
           static_workspace: bool = False, precond=None, precond_mode: Optional[str] = None):
    """Run the detector on device tensors.

    H (B, Nbs, K) and Y (B, Nbs, R): complex64 or complex128 CUDA tensors,
    contiguous, same dtype; sigma2 (B,) float64 CUDA tensor.  Returns
    (xhat (B, K, R) like H, labels (B, K, R) uint8, flags (B,) int32 bits).
    chan_idx (int32 CUDA tensor) restricts the launch to those channels;
    kappa (float32 CUDA tensor of B) receives per-channel condition-number
    estimates and gain (float32 CUDA tensor (B, K)) each user's effective
    gain, the input of demap_maxlog (fpcg_detect_ex).  static_workspace=True
    runs such launches through fpcg_detect_ex_static, which allocates
    nothing (its workspace is a fixed per-GPU array; calls that overlap on
    one GPU race).  schedule_=None runs the precision heuristic's format for
    the context's E{kappa} of the workload class.  precond (complex64 CUDA
    tensor (B, K, L) for FP32 work, complex128 for "fp64") keeps the
    block-Jacobi factor T across calls (fpcg_detect_pc): precond_mode
    "store" writes the factor this launch computes, "load" uses the given
    one in place of the block factorisation.
    """
    import torch

    if isinstance(schedule_, str):
        sched = schedule(schedule_, refresh_every, refine_steps, variant)
    else:
        sched = schedule_                       # a Schedule, or None: the heuristic's (fpcg_detect)
    if H.dtype not in (torch.complex64, torch.complex128) or Y.dtype != H.dtype:
        raise TypeError("H and Y must both be complex64 or both complex128")
    if not (H.is_cuda and Y.is_cuda and sigma2.is_cuda):
        raise TypeError("H, Y and sigma2 must be CUDA tensors")
    if sigma2.dtype != torch.float64:
        raise TypeError("sigma2 must be float64")
    H = H.contiguous()
    Y = Y.contiguous()
    sigma2 = sigma2.contiguous()
    B, Nbs, K = H.shape
    R = Y.shape[2]
    if Y.shape[:2] != (B, Nbs) or sigma2.shape != (B,):
        raise ValueError("shape mismatch between H, Y and sigma2")
    if Y.device != H.device or sigma2.device != H.device:
        raise TypeError("H, Y and sigma2 must be on the same device")
    dev = H.device.index or 0
    ctx = ctx or _ctx_for(dev)
    if out is None:
        xhat = torch.empty((B, K, R), dtype=H.dtype, device=H.device)
        labels = torch.empty((B, K, R), dtype=torch.uint8, device=H.device)
        flags = torch.empty((B,), dtype=torch.int32, device=H.device)
    else:
        xhat, labels, flags = out
        _check_tensor(xhat, "xhat", (B, K, R), H.dtype, H.device)
        _check_tensor(labels, "labels", (B, K, R), torch.uint8, H.device)
        _check_tensor(flags, "flags", (B,), torch.int32, H.device)
    if precond is not None or precond_mode is not None:
        if chan_idx is not None or kappa is not None or gain is not None or static_workspace:
            raise ValueError("precond does not combine with chan_idx, kappa, gain or static_workspace")
        if precond_mode not in ("store", "load") or precond is None or L <= 0 or sched is None:
            raise ValueError("precond needs L > 0, a schedule, a tensor and precond_mode 'store' or 'load'")
        work64 = sched is not None and sched.work == FMT["fp64"]
        _check_tensor(precond, "precond", (B, K, L), torch.complex128 if work64 else torch.complex64, H.device)
        _check(lib().fpcg_detect_pc(ctx.handle, _stream_handle(stream, H.device), B, Nbs, K, R,
                                    ctypes.c_void_p(H.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                    1 if H.dtype == torch.complex64 else 0, ctypes.c_void_p(sigma2.data_ptr()),
                                    qam, iters, L, ctypes.byref(sched) if sched is not None else None,
                                    ctypes.c_void_p(xhat.data_ptr()), ctypes.c_void_p(labels.data_ptr()),
                                    ctypes.c_void_p(flags.data_ptr()), ctypes.c_void_p(precond.data_ptr()),
                                    PRECOND_STORE if precond_mode == "store" else PRECOND_LOAD))
        return xhat, labels, flags
    if chan_idx is not None or kappa is not None or gain is not None or static_workspace:
        if chan_idx is not None:
            if chan_idx.dtype != torch.int32 or not chan_idx.is_cuda or chan_idx.device != H.device:
                raise TypeError("chan_idx must be an int32 CUDA tensor on the device of H")
        if kappa is not None:
            _check_tensor(kappa, "kappa", (B,), torch.float32, H.device)
        if gain is not None:
            _check_tensor(gain, "gain", (B, K), torch.float32, H.device)
        idx = chan_idx.contiguous() if chan_idx is not None else None
        entry = lib().fpcg_detect_ex_static if static_workspace else lib().fpcg_detect_ex
        _check(entry(ctx.handle, _stream_handle(stream, H.device), B, Nbs, K, R,
                                    ctypes.c_void_p(H.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                    1 if H.dtype == torch.complex64 else 0, ctypes.c_void_p(sigma2.data_ptr()),
                                    qam, iters, L, ctypes.byref(sched) if sched is not None else None,
                                    ctypes.c_void_p(xhat.data_ptr()), ctypes.c_void_p(labels.data_ptr()),
                                    ctypes.c_void_p(flags.data_ptr()),
                                    ctypes.c_void_p(idx.data_ptr() if idx is not None else 0),
                                    idx.numel() if idx is not None else 0,
                                    ctypes.c_void_p(kappa.data_ptr() if kappa is not None else 0),
                                    ctypes.c_void_p(gain.data_ptr() if gain is not None else 0)))
        return xhat, labels, flags
    _check(lib().fpcg_detect(ctx.handle, _stream_handle(stream, H.device), B, Nbs, K, R,
                             ctypes.c_void_p(H.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                             1 if H.dtype == torch.complex64 else 0, ctypes.c_void_p(sigma2.data_ptr()),
                             qam, iters, L, ctypes.byref(sched) if sched is not None else None,
                             ctypes.c_void_p(xhat.data_ptr()), ctypes.c_void_p(labels.data_ptr()),
                             ctypes.c_void_p(flags.data_ptr())))
    return xhat, labels, flags


def gram(H, Y, sigma2, schedule_: "str | Schedule" = "fp64", ctx: Optional[Context] = None, stream=None):
    """The Gram A = H^H H + sigma^2 I (B, K, K) and matched filter H^H Y
    (B, K, R) as the detector forms them for the schedule (fpcg_gram), in u_W:
    complex64 for reduced-precision schedules, complex128 for "fp64".
    Returns (A, Bmf, flags)."""
    import torch

    sched = schedule(schedule_) if isinstance(schedule_, str) else schedule_
    if H.dtype not in (torch.complex64, torch.complex128) or Y.dtype != H.dtype:
        raise TypeError("H and Y must both be complex64 or both complex128")
    if not (H.is_cuda and Y.is_cuda and sigma2.is_cuda) or sigma2.dtype != torch.float64:
        raise TypeError("H, Y: CUDA tensors; sigma2: float64 CUDA tensor")
    H, Y, sigma2 = H.contiguous(), Y.contiguous(), sigma2.contiguous()
    B, Nbs, K = H.shape
    if Y.dim() != 3 or Y.shape[:2] != (B, Nbs) or sigma2.shape != (B,):
        raise ValueError("shape mismatch between H, Y and sigma2")
    R = Y.shape[2]
    odt = torch.complex128 if sched.work == FMT["fp64"] else torch.complex64
    A = torch.empty((B, K, K), dtype=odt, device=H.device)
    Bm = torch.empty((B, K, R), dtype=odt, device=H.device)
    flags = torch.empty((B,), dtype=torch.int32, device=H.device)
    ctx = ctx or _ctx_for(H.device.index or 0)
    _check(lib().fpcg_gram(ctx.handle, _stream_handle(stream, H.device), B, Nbs, K, R,
                           ctypes.c_void_p(H.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                           1 if H.dtype == torch.complex64 else 0, ctypes.c_void_p(sigma2.data_ptr()),
                           ctypes.byref(sched), ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(Bm.data_ptr()),
                           ctypes.c_void_p(flags.data_ptr())))
    return A, Bm, flags


def slice_qam(x, qam: int, stream=None):
    """QAM slicer on a complex CUDA tensor; uint8 labels of the same shape."""
    import torch

    if not getattr(x, "is_cuda", False) or x.dtype not in (torch.complex64, torch.complex128):
        raise TypeError("x must be a complex64 or complex128 CUDA tensor")
    x = x.contiguous()
    labels = torch.empty(x.shape, dtype=torch.uint8, device=x.device)
    _check(lib().fpcg_slice(_stream_handle(stream, x.device), x.numel(), ctypes.c_void_p(x.data_ptr()),
                            1 if x.dtype == torch.complex64 else 0, qam, ctypes.c_void_p(labels.data_ptr())))
    return labels


def demap_maxlog(x, gain, qam: int, out=None, stream=None, scale=None):
    """Max-log LLRs (fpcg_demap_maxlog) of the estimates x (B, K, R) complex
    CUDA tensor with the detector's gains (B, K) float32: float32 tensor
    (B, K, R, log2 qam), most significant label bit first.  With `scale`, the
    LLRs as saturated int8 values round(LLR * scale) (fpcg_demap_maxlog_i8)."""
    import torch

    if not getattr(x, "is_cuda", False) or x.dtype not in (torch.complex64, torch.complex128) or x.dim() != 3:
        raise TypeError("x must be a complex64 or complex128 CUDA tensor (B, K, R)")
    x = x.contiguous()
    nb = {4: 2, 16: 4, 64: 6, 256: 8}.get(qam)
    if nb is None:
        raise ValueError(f"qam={qam}")
    if not getattr(gain, "is_cuda", False) or gain.device != x.device or gain.dtype != torch.float32 \
            or tuple(gain.shape) != tuple(x.shape[:2]):
        raise TypeError("gain must be a float32 CUDA tensor (B, K) on the device of x")
    gain = gain.contiguous()
    odt = torch.float32 if scale is None else torch.int8
    if out is None:
        llr = torch.empty(tuple(x.shape) + (nb,), dtype=odt, device=x.device)
    else:
        _check_tensor(out, "out", tuple(x.shape) + (nb,), odt, x.device)
        llr = out
    if scale is not None:
        _check(lib().fpcg_demap_maxlog_i8(_stream_handle(stream, x.device), x.numel(), x.shape[2],
                                          ctypes.c_void_p(x.data_ptr()), 1 if x.dtype == torch.complex64 else 0,
                                          ctypes.c_void_p(gain.data_ptr()), qam, float(scale),
                                          ctypes.c_void_p(llr.data_ptr())))
        return llr
    _check(lib().fpcg_demap_maxlog(_stream_handle(stream, x.device), x.numel(), x.shape[2],
                                   ctypes.c_void_p(x.data_ptr()), 1 if x.dtype == torch.complex64 else 0,
                                   ctypes.c_void_p(gain.data_ptr()), qam, ctypes.c_void_p(llr.data_ptr())))
    return llr


def round_operand(x, fmt: str, scale: float = 1.0, stream=None):
    """fl(.) of the detector's operand conversion on a float32 CUDA tensor."""
    import torch

    if not getattr(x, "is_cuda", False) or x.dtype != torch.float32:
        raise TypeError("x must be a float32 CUDA tensor")
    if fmt not in FMT:
        raise ValueError(f"unknown format {fmt!r}")
    x = x.contiguous()
    out = torch.empty_like(x)
    _check(lib().fpcg_round(_stream_handle(stream, x.device), x.numel(), ctypes.c_void_p(x.data_ptr()),
                            FMT[fmt], scale, ctypes.c_void_p(out.data_ptr())))
    return out


class Server:
    """Continuous-batching request loop over host buffers (fpcg_server_*)."""

    def __init__(self, ctx: Context, n_slots: int = 4, queue_cap: int = 1024):
        self.ctx = ctx
        self._h = ctypes.c_void_p()
        _check(lib().fpcg_server_create(ctx.handle, n_slots, queue_cap, ctypes.byref(self._h)))
        self._keep = {}
        self._chans = {}

    def channels(self, H, sigma2):
        """Upload a channel set (H (B, Nbs, K) complex64/complex128, sigma2 (B,))
        to the device once; returns a handle for submit(channels=...)."""
        import numpy as np

        H = np.ascontiguousarray(H)
        s2 = np.ascontiguousarray(sigma2, dtype=np.float64)
        B, Nbs, K = H.shape
        h = ctypes.c_uint64()
        _check(lib().fpcg_server_channels(self._h, B, Nbs, K, 1 if H.dtype == np.complex64 else 0,
                                          H.ctypes.data, s2.ctypes.data, ctypes.byref(h)))
        self._chans[h.value] = (B, Nbs, K, H.dtype)
        return h.value

    def release(self, handle):
        _check(lib().fpcg_server_release(self._h, handle))
        self._chans.pop(handle, None)

    def channels_update(self, handle, H, sigma2, keep_precond: bool = True):
        """Replace a channel set's H and sigma2 with the channels' next
        realisation (same shape and dtype); keep_precond keeps the block-Jacobi
        factors the set holds, so later requests precondition with them."""
        import numpy as np

        if handle not in self._chans:
            raise ValueError(f"unknown channel-set handle {handle}")
        B, Nbs, K, dt = self._chans[handle]
        H = np.ascontiguousarray(H)
        s2 = np.ascontiguousarray(sigma2, dtype=np.float64)
        if H.shape != (B, Nbs, K) or H.dtype != dt or s2.shape != (B,):
            raise ValueError(f"H must be {dt} of shape {(B, Nbs, K)} and sigma2 of shape ({B},)")
        _check(lib().fpcg_server_channels_update(self._h, handle, H.ctypes.data, s2.ctypes.data,
                                                 1 if keep_precond else 0))

    def submit(self, H, Y, sigma2, qam, iters, L=0, schedule_: "str | Schedule" = "fp64",
               refresh_every=0, refine_steps=0, variant=0, channels=None):
        """H, Y, sigma2: numpy arrays (complex64/complex128, float64); with
        `channels` (a handle from channels()) H and sigma2 may be None and only
        Y is sent.  Returns a ticket."""
        import numpy as np

        sched = schedule(schedule_, refresh_every, refine_steps, variant) if isinstance(schedule_, str) else schedule_
        # the library copies B*Nbs*R elements of Y (and B*Nbs*K of H, B of
        # sigma2) from these host arrays: every shape is checked here first
        if channels is not None:
            if channels not in self._chans:
                raise ValueError(f"unknown channel-set handle {channels}")
            B, Nbs, K, dt = self._chans[channels]
            Y = np.ascontiguousarray(Y, dtype=dt)
            H = s2 = None
            hp = sp = None
        else:
            H = np.ascontiguousarray(H)
            if H.dtype not in (np.complex64, np.complex128) or H.ndim != 3:
                raise TypeError("H must be a complex64 or complex128 array (B, Nbs, K)")
            Y = np.ascontiguousarray(Y, dtype=H.dtype)
            s2 = np.ascontiguousarray(sigma2, dtype=np.float64)
            B, Nbs, K = H.shape
            dt = H.dtype
            if s2.shape != (B,):
                raise ValueError(f"sigma2 must have shape ({B},), got {s2.shape}")
            hp, sp = H.ctypes.data, s2.ctypes.data
        if Y.ndim != 3 or Y.shape[:2] != (B, Nbs):
            raise ValueError(f"Y must have shape ({B}, {Nbs}, R), got {Y.shape}")
        R = Y.shape[2]
        xhat = np.empty((B, K, R), dtype=dt)
        labels = np.empty((B, K, R), dtype=np.uint8)
        flags = np.empty((B,), dtype=np.uint32)
        req = _Request(B, Nbs, K, R, 1 if dt == np.complex64 else 0, qam, iters, L, sched,
                       hp, Y.ctypes.data, sp, xhat.ctypes.data, labels.ctypes.data,
                       flags.ctypes.data, channels or 0)
        t = ctypes.c_uint64()
        _check(lib().fpcg_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = (H, Y, s2, xhat, labels, flags)
        return t.value

    def poll(self, ticket):
        """None while running, else (xhat, labels, flags)."""
        d = ctypes.c_int32()
        st = lib().fpcg_poll(self._h, ticket, ctypes.byref(d))
        if st != OK:
            self._keep.pop(ticket, None)
            _check(st)
        if not d.value:
            return None
        H, Y, s2, xhat, labels, flags = self._keep.pop(ticket)
        return xhat, labels, flags

    def drain(self):
        _check(lib().fpcg_drain(self._h))

    def stats(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
        _check(lib().fpcg_server_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def close(self):
        if self._h:
            lib().fpcg_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
