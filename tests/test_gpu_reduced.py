"""GPU parity of Reduced RCholeskyQR (Algorithm 5) against the FP64 oracle.

Z = (L X) R^{-1} depends on R exactly as Q = X R^{-1} does, so the bounds
follow the one-pass factorisation's: R within ~u n kappa of the oracle's
(same Theta, sums in another order), Z within ~u n kappa of its norm; the
FP32 and mixed paths round X's products at ~2^-24 (bf16 x 3 or the 24-bit
quantisation), so they get 2e-4 at kappa = 100.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def rq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_09953_amd as rq
    rq.lib()
    return rq


def _gpu(a):
    import torch
    import paper_2210_09953_amd as rq
    return rq.fortran(torch.from_numpy(np.asfortranarray(a)).to("cuda"))


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("m,n,k,l", [(20000, 40, 120, 30), (5001, 33, 99, 7)])
def test_reduced_f64_parity(rq, orc, kind, m, n, k, l):
    X = synth.make_x(m, n, 1e-6, seed=m + l)
    Z, R, ex = rq.reduced(_gpu(X), k, l, 13, kind=kind, want_s=True)
    assert rq.status(ex["ws"]) == 0
    ref = orc.reduced_rcholqr(X, k, l, 13, kind, want_s=True)
    kappa = np.linalg.cond(X / np.linalg.norm(X, axis=0))
    Z, R, S = _np(Z), _np(R), _np(ex["S"])
    assert np.linalg.norm(R - ref["R"]) <= 50 * U64 * n * kappa * np.linalg.norm(ref["R"])
    assert np.linalg.norm(Z - ref["Z"]) <= 50 * U64 * n * kappa * np.linalg.norm(ref["Z"])
    assert np.linalg.norm(S.T @ S - np.eye(n), 2) <= 100 * U64 * n
    assert np.array_equal(np.tril(R, -1), np.zeros((n, n))) and np.all(np.diag(R) > 0)


@pytest.mark.parametrize("precision", ["F32", "MIXED"])
def test_reduced_f32_and_mixed_parity(rq, orc, precision):
    import torch
    m, n, k, l = 60000, 64, 192, 64
    X32 = synth.make_x(m, n, 1e-2, seed=31, dtype=np.float32)
    Xg = _gpu(X32)
    Z, R = rq.reduced(Xg, k, l, 4, kind=rq.RADEMACHER, precision=getattr(rq, precision))
    Z2, R2 = rq.reduced(Xg, k, l, 4, kind=rq.RADEMACHER, precision=getattr(rq, precision))
    torch.cuda.synchronize()
    assert torch.equal(Z, Z2) and torch.equal(R, R2)  # deterministic
    ref = orc.reduced_rcholqr(X32.astype(np.float64), k, l, 4, orc.RADEMACHER)
    dZ = np.linalg.norm(_np(Z) - ref["Z"]) / np.linalg.norm(ref["Z"])
    dR = np.linalg.norm(_np(R) - ref["R"]) / np.linalg.norm(ref["R"])
    print(f"reduced {precision}: dZ={dZ:.2e} dR={dR:.2e}")
    assert dZ <= 2e-4 and dR <= 2e-4


def test_reduced_theta_part_is_the_factor_sketch(rq, orc):
    """The R of the reduced run is the R of Algorithm 2 with the same seed
    (same Theta rows; the sums differ only in their split order)."""
    m, n, k, l = 12000, 24, 72, 20
    X = synth.make_x(m, n, 1e-4, seed=3)
    Xg = _gpu(X)
    _, Rr = rq.reduced(Xg, k, l, 77, kind=rq.GAUSSIAN)
    _, R1 = rq.factor(Xg, k, 77, rq.GAUSSIAN, passes=1)
    Rr, R1 = _np(Rr), _np(R1)
    assert np.linalg.norm(Rr - R1) <= 1e-10 * np.linalg.norm(R1)
