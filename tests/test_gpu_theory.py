"""The paper's exactness result on the GPU path: under spatial orthogonality
(Assumption 2: different users' channel columns orthogonal, so the Gram is
block diagonal with one N_UE x N_UE block per user) and N_UE <= L, the
block-Jacobi-preconditioned matrix is the identity (Thm 5, App. D) and one
iteration of Alg. 3 returns the LMMSE solution."""
import sys

import numpy as np
import pytest

from oracle import detect as D

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _orthogonal_users(B, Nbs, K, n_ue, R, sigma2, seed):
    """H = U G: U (Nbs x K) with orthonormal columns, G = blockdiag of one
    random n_ue x n_ue matrix per user, so H^H H = G^H G is block diagonal."""
    rng = np.random.default_rng(seed)
    H = np.empty((B, Nbs, K), dtype=np.complex128)
    for c in range(B):
        U, _ = np.linalg.qr(rng.standard_normal((Nbs, K)) + 1j * rng.standard_normal((Nbs, K)))
        G = np.zeros((K, K), dtype=np.complex128)
        for u in range(K // n_ue):
            sl = slice(u * n_ue, (u + 1) * n_ue)
            G[sl, sl] = (rng.standard_normal((n_ue, n_ue)) + 1j * rng.standard_normal((n_ue, n_ue))) / np.sqrt(2)
        H[c] = U @ G
    Y = rng.standard_normal((B, Nbs, R)) + 1j * rng.standard_normal((B, Nbs, R))
    return H, Y, np.full(B, sigma2)


def _run(H, Y, s2, iters, L, sched, variant, io, kappa=False):
    import torch

    import paper_2504_09820_amd as fp

    dev = torch.device("cuda:0")
    Ht = torch.from_numpy(H.astype(io)).to(dev)
    Yt = torch.from_numpy(Y.astype(io)).to(dev)
    st = torch.from_numpy(s2).to(dev)
    kap = torch.empty((H.shape[0],), dtype=torch.float32, device=dev) if kappa else None
    x, _, fl = fp.detect(Ht, Yt, st, 16, iters, L, sched, variant=variant, kappa=kap)
    torch.cuda.synchronize()
    return (x.cpu().numpy().astype(np.complex128), fl.cpu().numpy(),
            None if kap is None else kap.cpu().numpy().astype(np.float64))


@pytest.mark.parametrize("L,variant", [(4, 0), (4, 1), (4, 2), (8, 0), (8, 2)])
def test_one_iteration_is_exact_under_spatial_orthogonality(L, variant):
    B, Nbs, K, n_ue, R = 12, 64, 32, 4, 5
    H, Y, s2 = _orthogonal_users(B, Nbs, K, n_ue, R, 0.05, seed=10 + L + variant)
    _say(f"case Thm 5 fp64 L={L} v{variant}")
    A, b = D.gram(H, Y, s2)
    x_exact = D.lmmse(A, b)
    x1, fl, kap = _run(H, Y, s2, 1, L, "fp64", variant, np.complex128, kappa=True)
    rel = np.linalg.norm(x1 - x_exact, axis=-2) / np.linalg.norm(x_exact, axis=-2)
    _say(f"  one iteration: max rel {rel.max():.2e}; kappa estimate {kap.min():.6f}..{kap.max():.6f}")
    assert np.all(fl == 0)
    assert rel.max() < 1e-12
    # the iteration matrix is I: its only Ritz value is 1
    np.testing.assert_allclose(kap, 1.0, atol=1e-5)
    # without a preconditioner one iteration is far from it (the users' blocks are not scaled)
    x0, _, _ = _run(H, Y, s2, 1, 0, "fp64", 0, np.complex128)
    rel0 = np.linalg.norm(x0 - x_exact, axis=-2) / np.linalg.norm(x_exact, axis=-2)
    assert np.median(rel0) > 1e-2


def test_one_iteration_fp16_symmetric_form():
    """The timed schedule (fp16 operands, symmetric form): after one iteration
    the error is that of rounding the identity-like matrix to fp16."""
    B, Nbs, K, n_ue, R = 12, 64, 32, 4, 5
    H, Y, s2 = _orthogonal_users(B, Nbs, K, n_ue, R, 0.05, seed=30)
    _say("case Thm 5 fp16 L=4 v2")
    A, b = D.gram(H, Y, s2)
    x_exact = D.lmmse(A, b)
    x1, fl, _ = _run(H, Y, s2, 1, 4, "fp16", 2, np.complex64)
    rel = np.linalg.norm(x1 - x_exact, axis=-2) / np.linalg.norm(x_exact, axis=-2)
    _say(f"  one iteration fp16: median rel {np.median(rel):.2e}, max {rel.max():.2e}")
    assert np.all(fl == 0)
    assert rel.max() < 2e-2                    # a few fp16 unit roundoffs times sqrt(K)
