"""Plain CPU oracle of the finite-precision (block-Jacobi) CG detector.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Shapes: a batch of B independent channels.  H (B, M, K), Y (B, M, R) complex;
every column of Y is an independent detection problem A x = b that shares A
with the other columns of its channel.  Scalars of the iterations (alpha,
beta, phi, rho) are per column, shaped (B, 1, R).

What is computed and where the paper defines it
  * gram():        A = H^H H + sigma^2 I and b = H^H y (eq. inversion and the
                   A_LMMSE definition in Sec. II).
  * lmmse():       x = A^{-1} b by Cholesky (the exact solve CG approximates).
  * cg_alg1():     Alg. 1 with alpha from eq. alpha (denominator r^H A p).
  * fp_cg():       Alg. 2 (FP-CG): A p at u_MV, inner products at u_IP, the
                   rest at u_W; alpha denominator p^H A p.
  * bj_inverse():  eq. pre_BJ: M_d = blockdiag(A_1^{-1}, ..., A_d^{-1}).
  * fp_bj_cg():    Alg. 3 (FP-BJ-CG), left-preconditioned, rho = r^H p for
                   alpha and for beta's denominator, z = M_d r, rho' = r^H z.
  * detect():      the full hot path: Gram/matched filter in the operand
                   format, the (P)CG solve with an optional FP64 residual
                   refresh, optional FP64 iterative refinement through H,
                   then the QAM slicer.
  * lanczos_kappa(): the condition number of the iteration matrix estimated
                   from the CG coefficients alpha_i, beta_i (the Lanczos
                   tridiagonal of CG, a textbook identity the paper does not
                   use; it feeds eq. heuristic / eq. heuristic_bj with a
                   per-channel kappa instead of E{kappa}).

Readings where the paper is silent:
  R-alpha  alpha and beta use the real parts of the inner products (A is
           Hermitian positive definite, the imaginary parts are rounding noise).
  R-guard  breakdown: if phi <= 0, rho <= 0 or either is not finite, that
           column is frozen from then on (alpha = beta = 0, x unchanged) and
           its channel is flagged.
  R-sched  the reduced-precision schedules: operands rounded to the operand format,
           products exact, each matrix product / inner product summed exactly
           and rounded once to the accumulation format (an idealised matrix
           core); u_W updates x, r, p use one rounding per fused multiply-add.
  R-fp8    fp8 e4m3 operands carry power-of-two scales: one per channel for
           H and for A, one per column for Y and for p.
  R-conv   H and y reach a reduced-precision operand format through fp32
           (rounded to fp32 first, then to the operand format).
  R-refr   FP64 refresh: every k iterations r <- b - A x in FP64 arithmetic on
           the stored Gram (k-th, 2k-th, ... iteration, not the last one).
  R-refi   FP64 refinement: r = H^H (y - H x) - sigma^2 x in FP64, scaled per
           column by a power of two to max|r| in [1, 2), solved with the same
           schedule and iteration count, and added to x in FP64.
  R-slice  per axis j = clamp(floor((v nu + m) / 2), 0, m - 1), nu =
           sqrt(2 (Q - 1) / 3), evaluated in the work precision; a tie goes to
           the upper level; label = (gray(j_I) << log2 m) | gray(j_Q).
"""
from __future__ import annotations

import dataclasses
import math
from fractions import Fraction

import numpy as np

from .rounding import fl, pow2_scale, round_real

# per-channel flag bits (same meaning on the GPU path)
FLAG_NONFINITE = 1
FLAG_BREAKDOWN = 2
FLAG_BLOCK_NOT_PD = 4
FLAG_FP8_SAT = 8


# --------------------------------------------------------------------------
# precision schedules
# --------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Schedule:
    """Which precision each step of the path runs in.

    gram_op : operand format of H and y in the Gram / matched filter
    mv_op   : u_MV, operand format of A and p in A p
    acc     : format the matrix products are accumulated / rounded to
    ip      : u_IP, inner products
    work    : u_W, every other step (alpha, beta, x, r, p, z updates)
    refresh_every : FP64 residual replacement period (0 = off)
    refine_steps  : FP64 iterative-refinement steps through H (0 = off)
    variant : 0 = Alg. 3 as printed (rho = r^H p); 1 = textbook PCG (rho = r^H z);
              2 = symmetric (split) form: Alg. 2 on T A T^H, x = T^H x_bar
    fma     : u_W updates of the form a*b + c rounded once (True) or twice
    accum   : "exact": every matrix / inner product is summed exactly and rounded
              once (an idealised matrix core); "sequential": the same sums as a
              chain of fused multiply-adds in the accumulation format, in index
              order; for fp8 operands, groups of 8 products summed with a
              truncating fixed-point alignment 13 bits below the group's
              largest product before each rounding (a second valid rounding
              order, used to measure how sensitive the iterates are to the
              order and granularity of rounding)
    """
    gram_op: str = "fp64"
    mv_op: str = "fp64"
    acc: str = "fp64"
    ip: str = "fp64"
    work: str = "fp64"
    refresh_every: int = 0
    refine_steps: int = 0
    variant: int = 0
    fma: bool = True
    accum: str = "exact"


FP64 = Schedule()
FP32 = Schedule("fp32", "fp32", "fp32", "fp32", "fp32")
BF16 = Schedule("bf16", "bf16", "fp32", "fp32", "fp32")
FP16 = Schedule("fp16", "fp16", "fp32", "fp32", "fp32")
FP8 = Schedule("e4m3", "e4m3", "fp32", "fp32", "fp32")

NAMED = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "fp16": FP16, "e4m3": FP8}


def schedule(name: str, **kw) -> Schedule:
    return dataclasses.replace(NAMED[name], **kw)


def paper_schedule(u_mv: str = "fp64", u_ip: str = "fp64", u_w: str = "fp64") -> Schedule:
    """Alg. 2 / Alg. 3 as the paper simulates them: the matrix-vector product's
    operands and result at u_MV, inner products at u_IP, everything else at u_W
    (A and b formed in u_W)."""
    return Schedule(gram_op=u_w, mv_op=u_mv, acc=u_mv, ip=u_ip, work=u_w, fma=False)


# --------------------------------------------------------------------------
# precision hooks used by the literal algorithms
# --------------------------------------------------------------------------
def _re(z):
    if isinstance(z, np.ndarray) and z.dtype == object:
        return np.vectorize(lambda v: v.real if hasattr(v, "real") else v, otypes=[object])(z)
    return np.real(z)


def _is_exact(a) -> bool:
    return isinstance(a, np.ndarray) and a.dtype == object


def _zeros(b):
    """x0 = 0 (exact zeros of b's kind; b * 0 would turn non-finite entries into nan)."""
    if _is_exact(b):
        return b * 0
    return np.zeros_like(b)


def _fma(a, b, c, fmt):
    """fl(a*b + c) with one rounding into fmt (a*b is exact in fp64 for operands
    of at most 26 significand bits; in fp64 itself this is two roundings)."""
    if fmt == "fp64":
        return a * b + c
    return round_real(a * b + c, fmt)


def _seq_dot_re(u, v, fmt):
    """Re(u^H v) over axis -2 as an ordered chain of fused multiply-adds."""
    ur, ui, vr, vi = np.real(u), np.imag(u), np.real(v), np.imag(v)
    s = np.zeros(u.shape[:-2] + (1, u.shape[-1]))
    for k in range(u.shape[-2]):
        s = _fma(ur[..., k:k + 1, :], vr[..., k:k + 1, :], s, fmt)
        s = _fma(ui[..., k:k + 1, :], vi[..., k:k + 1, :], s, fmt)
    return s


def _trunc_group_sum(terms, frac_bits):
    """Sum of a group of products aligned to the largest one: every product is
    truncated toward zero to a multiple of 2^(E - frac_bits), E the exponent of
    the largest |product| of the group, and the truncated values are added
    exactly."""
    mx = np.max(np.abs(terms), axis=0)
    _, e2 = np.frexp(np.where(mx > 0, mx, 1.0))
    q = np.ldexp(1.0, (e2 - 1 - frac_bits).astype(np.int64))
    return np.sum(np.trunc(terms / q) * q, axis=0)


def _seq_matmul_grouped(A, P, fmt, group=8, frac_bits=13):
    """A @ P (complex) accumulated group by group: 8 consecutive products of
    one real plane are summed with a truncating fixed-point alignment, then
    added to the accumulator with one rounding.  A valid rounding of the same
    sums whose error bound is that of an fp8 matrix core."""
    ar, ai, pr, pi = np.real(A), np.imag(A), np.real(P), np.imag(P)
    shp = A.shape[:-1] + (P.shape[-1],)
    wr = np.zeros(shp)
    wi = np.zeros(shp)
    K = A.shape[-1]
    for k0 in range(0, K, group):
        ks = range(k0, min(K, k0 + group))
        t_rr = np.stack([ar[..., :, k:k + 1] * pr[..., k:k + 1, :] for k in ks])
        t_ii = np.stack([-ai[..., :, k:k + 1] * pi[..., k:k + 1, :] for k in ks])
        t_ir = np.stack([ai[..., :, k:k + 1] * pr[..., k:k + 1, :] for k in ks])
        t_ri = np.stack([ar[..., :, k:k + 1] * pi[..., k:k + 1, :] for k in ks])
        wr = round_real(wr + _trunc_group_sum(t_rr, frac_bits), fmt)
        wr = round_real(wr + _trunc_group_sum(t_ii, frac_bits), fmt)
        wi = round_real(wi + _trunc_group_sum(t_ir, frac_bits), fmt)
        wi = round_real(wi + _trunc_group_sum(t_ri, frac_bits), fmt)
    return wr + 1j * wi


def _seq_matmul(A, P, fmt, grouped=False):
    """A @ P (complex) as ordered chains of real fused multiply-adds over k
    (grouped=True: the fp8 matrix-core style grouped accumulation)."""
    if grouped:
        return _seq_matmul_grouped(A, P, fmt)
    ar, ai, pr, pi = np.real(A), np.imag(A), np.real(P), np.imag(P)
    shp = A.shape[:-1] + (P.shape[-1],)
    wr = np.zeros(shp)
    wi = np.zeros(shp)
    for k in range(A.shape[-1]):
        a_r, a_i = ar[..., :, k:k + 1], ai[..., :, k:k + 1]
        p_r, p_i = pr[..., k:k + 1, :], pi[..., k:k + 1, :]
        wr = _fma(a_r, p_r, wr, fmt)
        wr = _fma(-a_i, p_i, wr, fmt)
        wi = _fma(a_i, p_r, wi, fmt)
        wi = _fma(a_r, p_i, wi, fmt)
    return wr + 1j * wi


class _Prec:
    """Rounding hooks for one schedule (identity in exact / fp64 mode)."""

    def __init__(self, sched: Schedule):
        self.s = sched

    def W(self, x):
        return x if _is_exact(x) else fl(x, self.s.work)

    def axpy(self, a, x, y):
        """u_W update y + a*x, fused (one rounding) or as two rounded ops."""
        if _is_exact(x) or self.s.work == "fp64":
            return y + a * x
        if self.s.fma:
            return fl(y + a * x, self.s.work)
        return fl(y + fl(a * x, self.s.work), self.s.work)

    def div(self, a, b):
        if _is_exact(a):
            return a / b
        with np.errstate(divide="ignore", invalid="ignore"):
            return fl(a / b, self.s.work)

    def ip(self, u, v):
        """Re(u^H v) per column at u_IP (exact sum, one rounding)."""
        if self.s.accum == "sequential" and not _is_exact(u):
            return _seq_dot_re(u, v, self.s.ip)
        d = _re(np.sum(np.conj(u) * v, axis=-2, keepdims=True))
        return d if _is_exact(d) else fl(d, self.s.ip)


class MatVec:
    """u_MV matrix-vector product w = A p for one schedule.

    The operand copy of A is made once (A_op = fl_MV(A), with a per-channel
    power-of-two scale for fp8); p is rounded to the operand format on every
    call (per-column scale for fp8); the product is summed exactly and rounded
    once to the accumulation format.
    """

    def __init__(self, A, sched: Schedule, flags=None):
        self.s = sched
        self.exact = _is_exact(A) or (sched.mv_op == "fp64" and sched.accum == "exact")
        self.sA = None
        if self.exact:
            self.A = A
            return
        if sched.mv_op == "fp64":
            self.A = A
            return
        if sched.mv_op == "e4m3":
            amax = np.max(np.maximum(np.abs(A.real), np.abs(A.imag)), axis=(-2, -1), keepdims=True)
            self.sA = pow2_scale(amax)
            self.A = fl(A * self.sA, "e4m3")
            if flags is not None:
                flags |= np.where(np.any(~np.isfinite(self.A), axis=(-2, -1)), FLAG_FP8_SAT, 0).astype(flags.dtype)
        else:
            self.sA = None
            self.A = fl(A, sched.mv_op)

    def _prod(self, A, P):
        if self.s.accum == "sequential":
            return _seq_matmul(A, P, self.s.acc, grouped=self.s.mv_op == "e4m3")
        return fl(A @ P, self.s.acc)

    def __call__(self, p):
        if self.exact:
            return self.A @ p
        if self.sA is not None:
            amax = np.max(np.maximum(np.abs(p.real), np.abs(p.imag)), axis=-2, keepdims=True)
            sp = pow2_scale(amax)
            pq = fl(p * sp, "e4m3")
            return self._prod(self.A, pq) / (self.sA * sp)
        return self._prod(self.A, fl(p, self.s.mv_op))


# --------------------------------------------------------------------------
# the plain definition
# --------------------------------------------------------------------------
def gram(H, Y, sigma2, sched: Schedule = FP64):
    """A = H^H H + sigma^2 I, b = H^H y (eq. inversion), in the schedule's formats.

    For sched.gram_op == "fp64" this is the plain definition.  Otherwise H and
    y are rounded to the operand format (fp8: per-channel scale for H, per
    column for y), the products are summed exactly and rounded once to the
    accumulation format, and sigma^2 is added to the rounded diagonal in u_W.
    """
    H = np.asarray(H)
    Y = np.asarray(Y)
    s2 = np.asarray(sigma2, dtype=np.float64).reshape(-1, 1, 1)
    K = H.shape[-1]
    eye = np.eye(K)
    if sched.gram_op == "fp64":
        Hh = np.conj(np.swapaxes(H, -1, -2))
        if sched.accum == "sequential":
            A = _hermitian_from_upper(_seq_matmul(Hh, H, "fp64")) + s2 * eye
            B = _seq_matmul(Hh, Y, "fp64")
            return A, B
        A = Hh @ H + s2 * eye
        B = Hh @ Y
        return A, B
    # R-conv: inputs reach the operand formats through fp32 (as the hardware
    # conversion instructions do)
    H = fl(H, "fp32")
    Y = fl(Y, "fp32")

    def prod(X, Z):
        if sched.accum == "sequential":
            return _seq_matmul(X, Z, sched.acc, grouped=sched.gram_op == "e4m3")
        return fl(X @ Z, sched.acc)

    if sched.gram_op == "e4m3":
        amax_h = np.max(np.maximum(np.abs(H.real), np.abs(H.imag)), axis=(-2, -1), keepdims=True)
        sh = pow2_scale(amax_h)
        amax_y = np.max(np.maximum(np.abs(Y.real), np.abs(Y.imag)), axis=-2, keepdims=True)
        sy = pow2_scale(amax_y)
        Hq = fl(H * sh, "e4m3")
        Yq = fl(Y * sy, "e4m3")
        Hh = np.conj(np.swapaxes(Hq, -1, -2))
        G = prod(Hh, Hq) / (sh * sh)
        B = prod(Hh, Yq) / (sh * sy)
    else:
        Hq = fl(H, sched.gram_op)
        Yq = fl(Y, sched.gram_op)
        Hh = np.conj(np.swapaxes(Hq, -1, -2))
        G = prod(Hh, Hq)
        B = prod(Hh, Yq)
    if sched.accum == "sequential":
        G = _hermitian_from_upper(G)
    A = G.copy()
    d = np.arange(K)
    A[:, d, d] = fl(G[:, d, d] + fl(s2[:, :, 0] + 0j, sched.work), sched.work)
    return A, B


def _hermitian_from_upper(G):
    """Upper triangle kept, lower = its conjugate transpose, real diagonal."""
    K = G.shape[-1]
    up = np.triu(np.ones((K, K), dtype=bool), 1)
    out = np.where(up, G, np.conj(np.swapaxes(G, -1, -2)))
    d = np.arange(K)
    out[..., d, d] = np.real(G[..., d, d])
    return out


def lmmse(A, B):
    """x = A^{-1} b by Cholesky A = C C^H and two triangular solves (FP64)."""
    import scipy.linalg as sla

    out = np.empty_like(B, dtype=np.complex128)
    for i in range(A.shape[0]):
        c = np.linalg.cholesky(A[i])
        t = sla.solve_triangular(c, B[i], lower=True)
        out[i] = sla.solve_triangular(c.conj().T, t, lower=False)
    return out


# --------------------------------------------------------------------------
# Alg. 1: CG detection
# --------------------------------------------------------------------------
def cg_alg1(A, b, iters: int, real_scalars: bool = True):
    """Alg. 1: r0 = b, p0 = r0, x0 = 0; alpha = r^H r / r^H A p (eq. alpha);
    x += alpha p (eq. update_of_x); r -= alpha A p (eq. update_of_r);
    beta = r_i^H r_i / r_{i-1}^H r_{i-1} (eq. beta); p = r + beta p (eq. update_of_p).
    Works for float and exact (Fraction object) arrays."""
    x = _zeros(b)
    r = b.copy()
    p = r.copy()

    def dot(u, v):
        d = np.sum(np.conj(u) * v, axis=-2, keepdims=True)
        return _re(d) if real_scalars else d

    for _ in range(iters):
        ap = A @ p
        rr = dot(r, r)
        alpha = rr / dot(r, ap)
        x = x + alpha * p
        r = r - alpha * ap
        beta = dot(r, r) / rr
        p = r + beta * p
    return x


# --------------------------------------------------------------------------
# Alg. 2: FP-CG and Alg. 3: FP-BJ-CG
# --------------------------------------------------------------------------
def _guard(phi, rho, live):
    """R-guard: a column stays live while phi > 0 and rho > 0 are finite."""
    if phi.dtype == object:
        ok = np.vectorize(lambda a, b: bool(a > 0 and b > 0), otypes=[bool])(phi, rho)
    else:
        with np.errstate(invalid="ignore"):
            ok = np.isfinite(phi) & np.isfinite(rho) & (phi > 0) & (rho > 0)
    return live & ok


def _select(mask, a, b):
    return np.where(mask, a, b)


def fp_cg(A, b, iters: int, sched: Schedule = FP64, mv=None, A_ref=None, trace=None, coeffs=None):
    """Alg. 2 (FP-CG).  Returns (x, broken) with broken a (B,) bool array.

    A is the Gram matrix in u_W (used for the FP64 refresh); ``mv`` is the u_MV
    product (defaults to MatVec(A, sched)); ``trace``, if a list, receives
    (x_i, r_i) after every iteration; ``coeffs``, if a list, receives
    (alpha_i, beta_i, live_i) after every iteration, each shaped (B, 1, R).
    """
    P = _Prec(sched)
    mv = mv if mv is not None else MatVec(A, sched)
    A_ref = A if A_ref is None else A_ref
    x = _zeros(b)
    r = b.copy()
    p = r.copy()
    live = np.ones(b.shape[:-2] + (1, b.shape[-1]), dtype=bool)
    broken = np.zeros(b.shape[0], dtype=bool)
    for i in range(1, iters + 1):
        w = mv(p)                                  # varpi = A p          [u_MV]
        phi = P.ip(p, w)                           # phi = p^H varpi      [u_IP]
        rho_prev = P.ip(r, r)                      # rho_{i-1} = r^H r    [u_IP]
        live_new = _guard(phi, rho_prev, live)
        broken |= np.any(live & ~live_new, axis=(-2, -1))
        live = live_new
        alpha = _select(live, P.div(rho_prev, phi), 0 * phi)   # [u_W]
        x = _select(live, P.axpy(alpha, p, x), x)              # x += alpha p
        r = _select(live, P.axpy(-alpha, w, r), r)             # r -= alpha varpi
        if sched.refresh_every and i % sched.refresh_every == 0 and i < iters:
            r = _select(live, P.W(b - A_ref @ x), r)           # R-refr: FP64 residual, rounded to u_W
        rho = P.ip(r, r)                                        # rho_i = r^H r
        beta = _select(live, P.div(rho, rho_prev), 0 * rho)     # beta = rho_i / rho_{i-1}
        p = _select(live, P.axpy(beta, p, r), p)               # p = r + beta p
        if trace is not None:
            trace.append((x.copy(), r.copy()))
        if coeffs is not None:
            coeffs.append((np.real(alpha).copy(), np.real(beta).copy(), live.copy()))
    return x, broken


def bj_factor(A, L: int, work: str = "fp64"):
    """T = blockdiag(C_1^{-1}, ..., C_d^{-1}) with A_i = C_i C_i^H (Cholesky), so
    that M_d = T^H T (eq. pre_BJ).  Computed in FP64 and rounded to ``work``.
    A block that is not numerically positive definite uses the inverse square
    root of its diagonal (flagged).  Returns (T, not_pd)."""
    Bn, K, _ = A.shape
    if K % L:
        raise ValueError("block size must divide K")
    T = np.zeros_like(A, dtype=np.complex128)
    not_pd = np.zeros(Bn, dtype=bool)
    for j in range(K // L):
        sl = slice(j * L, (j + 1) * L)
        for c in range(Bn):
            a = np.asarray(A[c, sl, sl], dtype=np.complex128)
            try:
                if not np.all(np.isfinite(a)):
                    raise np.linalg.LinAlgError
                import scipy.linalg as sla

                # C^{-1} by forward substitution: exactly lower triangular
                t = np.tril(sla.solve_triangular(np.linalg.cholesky(a), np.eye(L), lower=True))
                if not np.all(np.isfinite(t)):
                    raise np.linalg.LinAlgError
            except np.linalg.LinAlgError:
                not_pd[c] = True
                dg = np.real(np.diag(a))
                ok = np.isfinite(dg) & (dg > 0)
                t = np.diag(np.where(ok, 1.0 / np.sqrt(np.where(ok, dg, 1.0)), 1.0)).astype(np.complex128)
            T[c, sl, sl] = t
    return fl(T, work), not_pd


def split_system(A, T, work: str = "fp64"):
    """A_bar = T A T^H (the symmetrically preconditioned Gram of Thm 4), formed
    in FP64 from the u_W operands and rounded once to u_W; the upper triangle
    is kept and mirrored so that A_bar is exactly Hermitian."""
    Th = np.conj(np.swapaxes(T, -1, -2))
    Ab = T @ A @ Th
    K = A.shape[-1]
    up = np.triu(np.ones((K, K), dtype=bool), 1)
    Ab = np.where(up, Ab, np.conj(np.swapaxes(Ab, -1, -2)))
    d = np.arange(K)
    Ab[..., d, d] = np.real(Ab[..., d, d])
    return fl(Ab, work)


def bj_inverse(A, L: int, work: str = "fp64"):
    """eq. pre_BJ: M_d = blockdiag(A_1^{-1}, ..., A_d^{-1}) with L x L blocks.

    Each block is inverted through its Cholesky factor, A_i^{-1} = C^{-H} C^{-1}
    (computed in FP64 and rounded to ``work``).  A block that is not numerically
    positive definite falls back to the inverse of its diagonal (flagged).
    Returns (M (B, K, K), not_pd (B,) bool).
    """
    Bn, K, _ = A.shape
    if K % L:
        raise ValueError("block size must divide K")
    d = K // L
    M = np.zeros_like(A, dtype=np.complex128)
    not_pd = np.zeros(Bn, dtype=bool)
    for j in range(d):
        sl = slice(j * L, (j + 1) * L)
        blk = np.asarray(A[:, sl, sl], dtype=np.complex128)
        for c in range(Bn):
            a = blk[c]
            try:
                if not np.all(np.isfinite(a)):
                    raise np.linalg.LinAlgError
                ch = np.linalg.cholesky(a)
                ci = np.linalg.inv(ch)          # triangular inverse C^{-1}
                inv = ci.conj().T @ ci          # C^{-H} C^{-1}
                if not np.all(np.isfinite(inv)):
                    raise np.linalg.LinAlgError
            except np.linalg.LinAlgError:
                not_pd[c] = True
                dg = np.real(np.diag(a))
                ok = np.isfinite(dg) & (dg > 0)
                inv = np.diag(np.where(ok, 1.0 / np.where(ok, dg, 1.0), 1.0)).astype(np.complex128)
            M[c, sl, sl] = inv
    return fl(M, work), not_pd


def fp_bj_cg(A, b, iters: int, L: int, sched: Schedule = FP64, mv=None, M=None, A_ref=None, trace=None,
             coeffs=None):
    """Alg. 3 (FP-BJ-CG), left-preconditioned.  Returns (x, broken).

    variant 0 follows the printed algorithm (rho_{i-1} = r^H p for alpha and for
    beta's denominator); variant 1 is textbook PCG (rho = r^H z carried over);
    variant 2 is the symmetric (split) form: Alg. 2 on A_bar = T A T^H with
    b_bar = T b and x = T^H x_bar, T = blockdiag(C_i^{-1}) -- the system
    Thm 4 analyses; in exact arithmetic all three give the same iterates.
    """
    if sched.variant == 2:
        return fp_bj_cg_split(A, b, iters, L, sched, A_ref=A_ref, trace=trace, coeffs=coeffs)[:2]
    P = _Prec(sched)
    mv = mv if mv is not None else MatVec(A, sched)
    if M is None:
        M, _ = bj_inverse(A, L, sched.work if not _is_exact(A) else "fp64")
    A_ref = A if A_ref is None else A_ref
    x = _zeros(b)
    r = b.copy()
    p = P.W(M @ r)                                 # p0 = M_d r0            [u_W]
    rho_carry = P.ip(r, p)                         # textbook variant: r0^H z0
    live = np.ones(b.shape[:-2] + (1, b.shape[-1]), dtype=bool)
    broken = np.zeros(b.shape[0], dtype=bool)
    for i in range(1, iters + 1):
        w = mv(p)                                  # varpi = A p            [u_MV]
        phi = P.ip(p, w)                           # phi = p^H varpi        [u_IP]
        rho_prev = P.ip(r, p) if sched.variant == 0 else rho_carry   # rho = r^H p   [u_IP]
        live_new = _guard(phi, rho_prev, live)
        broken |= np.any(live & ~live_new, axis=(-2, -1))
        live = live_new
        alpha = _select(live, P.div(rho_prev, phi), 0 * phi)
        x = _select(live, P.axpy(alpha, p, x), x)
        r = _select(live, P.axpy(-alpha, w, r), r)
        if sched.refresh_every and i % sched.refresh_every == 0 and i < iters:
            r = _select(live, P.W(b - A_ref @ x), r)
        z = P.W(M @ r)                             # z = M_d r              [u_W]
        rho = P.ip(r, z)                           # rho_i = r^H z          [u_IP]
        beta = _select(live, P.div(rho, rho_prev), 0 * rho)
        p = _select(live, P.axpy(beta, p, z), p)   # p = z + beta p
        rho_carry = rho
        if trace is not None:
            trace.append((x.copy(), r.copy()))
        if coeffs is not None:
            coeffs.append((np.real(alpha).copy(), np.real(beta).copy(), live.copy()))
    return x, broken


# --------------------------------------------------------------------------
# QAM slicer and bit errors
# --------------------------------------------------------------------------
def fp_bj_cg_split(A, b, iters: int, L: int, sched: Schedule = FP64, T=None, Abar=None, mv=None, A_ref=None,
                   trace=None, coeffs=None):
    """Alg. 3 in its symmetric form: CG (Alg. 2 steps) on A_bar x_bar = b_bar,
    then x = T^H x_bar.  Returns (x, broken, T, A_bar)."""
    W = sched.work if not _is_exact(A) else "fp64"
    if T is None:
        T, _ = bj_factor(A, L, W)
    if Abar is None:
        Abar = split_system(A, T, W)
    mv = mv if mv is not None else MatVec(Abar, sched)
    bb = fl(T @ b, W) if not _is_exact(b) else T @ b
    xb, broken = fp_cg(Abar, bb, iters, sched, mv=mv, A_ref=Abar, trace=trace, coeffs=coeffs)
    Th = np.conj(np.swapaxes(T, -1, -2))
    x = fl(Th @ xb, W) if not _is_exact(xb) else Th @ xb
    return x, broken, T, Abar


def lanczos_tridiagonal(alphas, betas):
    """The Lanczos tridiagonal of m CG steps of one column (textbook identity,
    e.g. Saad, Iterative Methods for Sparse Linear Systems, Sec. 6.7.3): with
    the coefficients alpha_1..alpha_m (step sizes) and beta_1..beta_m (the
    ratios rho_i / rho_{i-1}),
        T[0, 0] = 1 / alpha_1,
        T[i, i] = 1 / alpha_{i+1} + beta_i / alpha_i          (i = 1..m-1),
        T[i-1, i] = T[i, i-1] = sqrt(beta_i) / alpha_i        (i = 1..m-1).
    The eigenvalues of T (Ritz values) approximate those of the iteration
    matrix (A; M_d A for the left-preconditioned Alg. 3; A_bar for its
    symmetric form) and lie inside its spectrum."""
    a = np.asarray(alphas, dtype=np.float64)
    bt = np.asarray(betas, dtype=np.float64)
    m = a.size
    T = np.zeros((m, m))
    T[0, 0] = 1.0 / a[0]
    for i in range(1, m):
        T[i, i] = 1.0 / a[i] + bt[i - 1] / a[i - 1]
        T[i - 1, i] = T[i, i - 1] = math.sqrt(bt[i - 1]) / a[i - 1]
    return T


def lanczos_kappa(coeffs, R_valid=None):
    """Per channel: the largest, over its received-vector columns, of
    lambda_max(T) / lambda_min(T) with T the Lanczos tridiagonal of the
    column's CG steps taken before any breakdown (coeffs from fp_cg /
    fp_bj_cg / detect).  A column without a step gives no estimate; a
    channel without any estimate gets NaN.  Each column's ratio is at most
    the iteration matrix's condition number (the Ritz values interlace)."""
    if not coeffs:
        raise ValueError("no CG steps recorded")
    al = np.stack([c[0] for c in coeffs], axis=0)[:, :, 0, :]     # (I, B, R)
    be = np.stack([c[1] for c in coeffs], axis=0)[:, :, 0, :]
    lv = np.stack([c[2] for c in coeffs], axis=0)[:, :, 0, :]
    I, Bn, R = al.shape
    R_valid = R if R_valid is None else R_valid
    out = np.full(Bn, np.nan)
    for ch in range(Bn):
        best = np.nan
        for j in range(R_valid):
            m = 0
            while m < I and lv[m, ch, j] and al[m, ch, j] > 0:
                m += 1
            if m == 0:
                continue
            # the last step's beta only enters through a further step
            ev = np.linalg.eigvalsh(lanczos_tridiagonal(al[:m, ch, j], be[:m, ch, j]))
            k = ev[-1] / ev[0] if ev[0] > 0 else np.inf
            best = k if np.isnan(best) else max(best, k)
        out[ch] = best
    return out


def _gray(n):
    return n ^ (n >> 1)


def slice_qam(xhat, q: int, work: str = "fp64"):
    """R-slice: nearest unit-energy square-QAM point, Gray label per axis.

    The decision is evaluated in ``work`` precision (fp32: numpy float32
    arithmetic, each operation rounded), so identical inputs give identical
    labels on any IEEE machine.
    """
    m = int(round(math.sqrt(q)))
    bits = m.bit_length() - 1
    dt = np.float32 if work == "fp32" else np.float64
    nu = dt(math.sqrt(2.0 * (q - 1) / 3.0))
    mm = dt(m)

    def axis(v):
        v = np.asarray(v, dtype=dt)
        with np.errstate(invalid="ignore", over="ignore"):
            t = (v * nu) + mm                     # two rounded operations
            j = np.floor(t * dt(0.5))
        j = np.where(np.isfinite(j), j, 0.0)
        j = np.clip(j, 0, m - 1).astype(np.int64)
        return j

    ji = axis(np.real(xhat))
    jq = axis(np.imag(xhat))
    return (_gray(ji) << bits) | _gray(jq)


def bit_errors(a, b) -> int:
    x = np.bitwise_xor(np.asarray(a, dtype=np.int64), np.asarray(b, dtype=np.int64))
    cnt = 0
    while np.any(x):
        cnt += int(np.sum(x & 1))
        x = x >> 1
    return cnt


# --------------------------------------------------------------------------
# the whole hot path
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Result:
    xhat: np.ndarray       # (B, K, R) complex128
    labels: np.ndarray     # (B, K, R) int64
    flags: np.ndarray      # (B,) uint32
    A: np.ndarray          # Gram in u_W
    b: np.ndarray          # matched filter in u_W


def detect(H, Y, sigma2, q: int, iters: int, L: int = 0, sched: Schedule = FP64, coeffs=None, T_given=None) -> Result:
    """Gram + matched filter -> (BJ setup) -> (P)CG -> (refinement) -> slicer.

    ``coeffs``, if a list, receives the CG coefficients of the first solve
    (the one of b; see fp_cg).  ``T_given`` (B, K, K), if set with L > 0,
    is the block-Jacobi factor T = blockdiag(C_i^{-1}) used in place of the
    factorisation of this A: a factor kept from earlier channel realisations
    (Sec. V, time-varying channel; eq. pre_BJ with the stored factor).  The
    preconditioner is then M_d = T^H T (formed in FP64, rounded once to u_W)
    or the symmetric form's T A T^H, and no block is flagged."""
    H = np.asarray(H, dtype=np.complex128)
    Y = np.asarray(Y, dtype=np.complex128)
    Bn = H.shape[0]
    flags = np.zeros(Bn, dtype=np.uint32)
    A, b = gram(H, Y, sigma2, sched)
    nonfin = ~(np.all(np.isfinite(A), axis=(-2, -1)) & np.all(np.isfinite(b), axis=(-2, -1)))
    flags |= np.where(nonfin, FLAG_NONFINITE, 0).astype(np.uint32)
    M = T = Abar = None
    split = bool(L) and sched.variant == 2
    if L:
        if T_given is not None:
            T = np.asarray(T_given, dtype=np.complex128)
            not_pd = np.zeros(Bn, dtype=bool)
            if not split:
                M = fl(np.conj(np.swapaxes(T, -1, -2)) @ T, sched.work)
        elif split:
            T, not_pd = bj_factor(A, L, sched.work)
        else:
            M, not_pd = bj_inverse(A, L, sched.work)
        if split:
            Abar = split_system(A, T, sched.work)
        flags |= np.where(not_pd, FLAG_BLOCK_NOT_PD, 0).astype(np.uint32)
    mv = MatVec(Abar if split else A, sched, flags)

    def solve(rhs, exact_back=False, coeffs=None):
        if split:
            bb = fl(T @ rhs, sched.work)
            xb, broken = fp_cg(Abar, bb, iters, sched, mv=mv, coeffs=coeffs)
            x = np.conj(np.swapaxes(T, -1, -2)) @ xb
            return (x if exact_back else fl(x, sched.work)), broken
        if L:
            return fp_bj_cg(A, rhs, iters, L, sched, mv=mv, M=M, coeffs=coeffs)
        return fp_cg(A, rhs, iters, sched, mv=mv, coeffs=coeffs)

    x, broken = solve(b, coeffs=coeffs)
    flags |= np.where(broken, FLAG_BREAKDOWN, 0).astype(np.uint32)
    slice_prec = sched.work
    if sched.refine_steps:
        x = x.astype(np.complex128)
        s2 = np.asarray(sigma2, dtype=np.float64).reshape(-1, 1, 1)
        Hh = np.conj(np.swapaxes(H, -1, -2))
        def solve_split_fp64(r):
            bb = fl(T @ r, sched.work)
            xb, broken = fp_cg(Abar, bb, iters, sched, mv=mv)
            return np.conj(np.swapaxes(T, -1, -2)) @ xb, broken    # x = T^H x_bar in FP64

        for _ in range(sched.refine_steps):
            res = Hh @ (Y - H @ x) - s2 * x                 # FP64, exact A
            amax = np.max(np.maximum(np.abs(res.real), np.abs(res.imag)), axis=-2, keepdims=True)
            sc = 1.0 / _pow2_floor(amax)
            if split:
                # b_bar = T (r sc) formed in FP64 from the u_W factor and rounded once
                d, broken = solve_split_fp64(res * sc)
            else:
                d, broken = solve(fl(res * sc, sched.work))
            flags |= np.where(broken, FLAG_BREAKDOWN, 0).astype(np.uint32)
            x = x + d.astype(np.complex128) / sc
        slice_prec = "fp64"
    labels = slice_qam(x, q, slice_prec)
    return Result(xhat=x, labels=labels, flags=flags, A=A, b=b)


def _pow2_floor(a):
    """2^floor(log2 a) for a > 0 finite, else 1."""
    a = np.asarray(a, dtype=np.float64)
    out = np.ones_like(a)
    ok = np.isfinite(a) & (a > 0)
    _, e2 = np.frexp(a[ok])
    out[ok] = np.ldexp(1.0, np.clip(e2.astype(np.int64) - 1, -126, 126))
    return out


def fraction_matrix(a) -> np.ndarray:
    """Helper for exact-arithmetic tests: object array of Fractions."""
    return np.vectorize(lambda v: Fraction(v), otypes=[object])(np.asarray(a))
