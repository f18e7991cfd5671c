"""A priori error bounds for the fp8 (e4m3) operand path, independent of any
model of how the matrix cores order or truncate their sums.

Thm 1 (complex-valued matrix computations) bounds a product computed in
precision u by gamma_2n-type terms.  Here the operands are rounded once to
e4m3 (Def. 1: relative error at most u = 2^-4, or half the subnormal spacing
2^-10 of the scaled value below the normal range) and the products are
accumulated in FP32 (u_acc = 2^-24).  Elementwise, for the Gram
    |A_gpu - A|_ij <= sum_k (|dh_ki||h_kj| + |h_ki||dh_kj| + |dh_ki||dh_kj|)
                      + sqrt(2) gamma_2Nbs(u_acc) ||h~_i|| ||h~_j|| (+ the FP32 rounding of sigma^2 + a_ii)
with |dh| the complex operand rounding bound, A the exact Gram of the
(complex64) inputs.  For A p, the product is not an output: it is checked
through phi = p^H (A p) of the first iteration (x_1 = alpha p_0, alpha =
r_0^H r_0 / phi, p_0 = r_0 = b), against the exact p^H A p of the GPU's own
Gram and matched filter, with the same operand and accumulation terms.
The fp8 parity cases' shapes are covered (K = 32, 64, 100, 120, 128).
"""
import math

import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu

U8 = 2.0**-4          # e4m3 unit roundoff (Def. 1, Table I extended)
SUB8 = 2.0**-10       # half the e4m3 subnormal spacing 2^-9
UACC = 2.0**-24       # FP32 accumulation


def gamma(n, u):
    return n * u / (1 - n * u)


def _pow2_scale(amax):
    """2^floor(log2(448 / amax)): the power-of-two scale the path's definition uses."""
    return 2.0 ** np.floor(np.log2(448.0 / amax))


def _rounding_bound(v, s):
    """Per complex element: bound on |fl8(v s)/s - v| (both components)."""
    def comp(x):
        return np.maximum(U8 * np.abs(x), SUB8 / s)
    return np.sqrt(comp(v.real) ** 2 + comp(v.imag) ** 2)


CASES = [(32, 128, 14, np.complex64), (64, 256, 14, np.complex64), (128, 512, 14, np.complex64),
         (100, 300, 17, np.complex128), (120, 300, 9, np.complex64)]


@pytest.mark.parametrize("K,Nbs,R,io", CASES, ids=[f"K{c[0]}-N{c[1]}-R{c[2]}" for c in CASES])
def test_fp8_gram_and_first_matvec_within_a_priori_bounds(K, Nbs, R, io):
    import torch

    import paper_2504_09820_amd as fp

    print(f"case fp8 bound K={K} Nbs={Nbs} R={R} io={np.dtype(io).name}", flush=True)
    wl = W.draw(4, Nbs, K, R, 64, 20.0, 0.5, 0.5, seed=91 + K)
    dev = torch.device("cuda:0")
    Ht = torch.from_numpy(wl.H.astype(io)).to(dev)
    Yt = torch.from_numpy(wl.Y.astype(io)).to(dev)
    st = torch.from_numpy(wl.sigma2).to(dev)
    A_g, B_g, fl = fp.gram(Ht, Yt, st, "fp8")
    x1, _, _ = fp.detect(Ht, Yt, st, 64, 1, 0, "fp8")
    torch.cuda.synchronize()
    A_g = A_g.cpu().numpy().astype(np.complex128)
    B_g = B_g.cpu().numpy().astype(np.complex128)
    x1 = x1.cpu().numpy().astype(np.complex128)
    assert not fl.cpu().numpy().any()
    # inputs as the path reads them (complex128 inputs reach e4m3 through fp32)
    H = wl.H.astype(io).astype(np.complex64).astype(np.complex128)
    Y = wl.Y.astype(io).astype(np.complex64).astype(np.complex128)
    for c in range(H.shape[0]):
        h = H[c]
        s = _pow2_scale(np.max(np.maximum(np.abs(h.real), np.abs(h.imag))))
        dh = _rounding_bound(h, s)
        ah = np.abs(h)
        A = h.conj().T @ h + wl.sigma2[c] * np.eye(K)
        nrm = np.linalg.norm(np.abs(h) + dh, axis=0)
        bound = dh.T @ ah + ah.T @ dh + dh.T @ dh + math.sqrt(2) * gamma(2 * Nbs, UACC) * np.outer(nrm, nrm)
        bound += np.diag(2 * UACC * np.abs(np.diag(A)))
        err = np.abs(A_g[c] - A)
        ratio = float(np.max(err / bound))
        print(f"  channel {c}: Gram max |err|/bound {ratio:.3f}, max |err| {err.max():.2e}", flush=True)
        assert np.all(err <= bound), ratio
        off = np.kron(1 - np.eye((K + 15) // 16), np.ones((16, 16)))[:K, :K].astype(bool)
        assert np.array_equal(A_g[c][off], A_g[c].conj().T[off])   # tiles below the diagonal mirrored
        # matched filter: the same bound with y's per-column scales
        y = Y[c]
        sy = _pow2_scale(np.max(np.maximum(np.abs(y.real), np.abs(y.imag)), axis=0))
        dy = _rounding_bound(y, sy[None, :])
        Bx = h.conj().T @ y
        ny = np.linalg.norm(np.abs(y) + dy, axis=0)
        bb = dh.T @ np.abs(y) + ah.T @ dy + dh.T @ dy + math.sqrt(2) * gamma(2 * Nbs, UACC) * np.outer(nrm, ny)
        assert np.all(np.abs(B_g[c] - Bx) <= bb)
        # first iteration: phi = p^H fl(A~ p~) with p = b (the GPU's own B), A the GPU's own Gram
        Ag, p = A_g[c], B_g[c]
        sA = _pow2_scale(np.max(np.maximum(np.abs(Ag.real), np.abs(Ag.imag))))
        sp = _pow2_scale(np.max(np.maximum(np.abs(p.real), np.abs(p.imag)), axis=0))
        dA = _rounding_bound(Ag, sA)
        dp = _rounding_bound(p, sp[None, :])
        nA = np.linalg.norm(np.abs(Ag) + dA, axis=1)
        npp = np.linalg.norm(np.abs(p) + dp, axis=0)
        w_bound = dA @ np.abs(p) + np.abs(Ag) @ dp + dA @ dp + math.sqrt(2) * gamma(2 * K, UACC) * np.outer(nA, npp)
        w = Ag @ p
        phi_ex = np.real(np.sum(np.conj(p) * w, axis=0))
        phi_bound = np.sum(np.abs(p) * w_bound, axis=0) + \
            math.sqrt(2) * gamma(2 * K, UACC) * np.linalg.norm(p, axis=0) * np.linalg.norm(np.abs(w) + w_bound, axis=0)
        rho = np.real(np.sum(np.conj(p) * p, axis=0))
        alpha = np.real(np.sum(np.conj(p) * x1[c], axis=0)) / rho          # x_1 = alpha p_0
        phi_g = rho / alpha
        # rho and alpha themselves carry FP32 roundings (u_IP = u_W = FP32)
        slack = phi_ex * 4 * gamma(2 * K + 4, UACC)
        dev_phi = np.abs(phi_g - phi_ex)
        print(f"  channel {c}: phi max |err|/bound {float(np.max(dev_phi / (phi_bound + slack))):.3f}", flush=True)
        assert np.all(dev_phi <= phi_bound + slack)
