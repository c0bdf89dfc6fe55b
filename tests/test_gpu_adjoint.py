"""GPU adjoint of the 2-pass factorisation against the FP64 oracle's closed
form (tests/test_oracle_pins.py pins it against finite differences and
autograd of LAPACK's QR), against finite differences of the GPU forward,
and through torch.autograd."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("m,n,kind", [(3000, 24, 0), (2001, 16, 1), (777, 50, 2), (1000, 1, 0),
                                      (2500, 20, 3)])
def test_backward_matches_oracle_f64(rq, orc, m, n, kind):
    X = synth.make_x(m, n, 1e-3, seed=11)
    dQ, dR = synth.make_cotangents(m, n, seed=12)
    Q, R, ex = rq.factor(_gpu(X), 3 * n, 5, kind, passes=2, want_factors=True)
    dX = _np(rq.backward(_gpu(X), ex["Rs"], ex["Rp"], _gpu(dQ), _gpu(dR)))
    ref = orc.rcholqr(X, 3 * n, 5, kind, passes=2)
    dXr = orc.qr_backward(ref["Q"], ref["R"], dQ, dR)
    err = np.linalg.norm(dX - dXr) / np.linalg.norm(dXr)
    print(f"adjoint f64 m={m} n={n}: rel err {err:.2e}")
    assert err <= 1e-10


def test_backward_matches_finite_differences_f64(rq):
    """m=2000, n=16, sigma 1 -> 1e-2, Gaussian: central differences of the
    GPU forward in FP64 against the GPU adjoint."""
    m, n, k = 2000, 16, 48
    X = synth.make_x(m, n, 1e-2, seed=13)
    dQ, dR = synth.make_cotangents(m, n, seed=14)

    def loss(Xn):
        Q, R = rq.factor(_gpu(Xn), k, 7, rq.GAUSSIAN, passes=2)
        return float(np.sum(_np(Q) * dQ) + np.sum(_np(R) * dR))

    _, _, ex = rq.factor(_gpu(X), k, 7, rq.GAUSSIAN, passes=2, want_factors=True)
    dX = _np(rq.backward(_gpu(X), ex["Rs"], ex["Rp"], _gpu(dQ), _gpu(dR)))
    E = np.asfortranarray(np.random.default_rng(15).standard_normal((m, n)))
    h = 1e-5 * np.linalg.norm(X) / np.linalg.norm(E)
    fd = (loss(X + h * E) - loss(X - h * E)) / (2 * h)
    an = float(np.sum(dX * E))
    print(f"FD {fd:.12e} adjoint {an:.12e}")
    assert abs(fd - an) <= 1e-6 * abs(an)


@pytest.mark.parametrize("precision", [1, 2])
def test_backward_f32_against_oracle(rq, orc, precision):
    """FP32 adjoint (configuration E shape scaled down: n=128, kappa=1e3)."""
    m, n, k = 60000, 128, 384
    X32 = synth.make_x(m, n, 1e-3, seed=16, dtype=np.float32)
    dQ, dR = synth.make_cotangents(m, n, seed=17)
    dQ32 = dQ.astype(np.float32)
    Q, R, ex = rq.factor(_gpu(X32), k, 3, rq.RADEMACHER, passes=2, precision=precision,
                         want_factors=True)
    dX = _np(rq.backward(_gpu(X32), ex["Rs"], ex["Rp"], _gpu(dQ32), _gpu(dR),
                         precision=precision)).astype(np.float64)
    X = X32.astype(np.float64)
    ref = orc.rcholqr(X, k, 3, orc.RADEMACHER, passes=2)
    dXr = orc.qr_backward(ref["Q"], ref["R"], dQ32.astype(np.float64), dR)
    err = np.linalg.norm(dX - dXr) / np.linalg.norm(dXr)
    print(f"adjoint precision={precision}: rel err vs FP64 oracle {err:.2e}")
    assert err <= 1e-3


def test_backward_zero_cotangent_and_deterministic_forward(rq):
    """The adjoint recomputes Q with the forward kernels; with dQ = dR = 0
    the product Q N vanishes, so check the recompute through a zero N:
    dX = Q N R^-T = 0 exactly, and a second factor call reproduces Q."""
    import torch
    m, n = 5000, 32
    X = _gpu(synth.make_x(m, n, 1e-4, seed=18, dtype=np.float32))
    Q1, R1, ex = rq.factor(X, 96, 2, rq.RADEMACHER, passes=2, want_factors=True)
    Q2, R2 = rq.factor(X, 96, 2, rq.RADEMACHER, passes=2)
    torch.cuda.synchronize()
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2)
    dX = rq.backward(X, ex["Rs"], ex["Rp"], torch.zeros_like(X), None)
    torch.cuda.synchronize()
    assert float(dX.abs().max()) == 0.0


def test_autograd_function(rq):
    import torch
    m, n = 4000, 20
    Xn = synth.make_x(m, n, 1e-2, seed=19)
    dQ, dR = synth.make_cotangents(m, n, seed=20)
    X = _gpu(Xn).requires_grad_(True)
    Q, R = rq.rcholqr2(X, 60, 4, rq.GAUSSIAN)
    loss = (Q * _gpu(dQ)).sum() + (R * _gpu(dR)).sum()
    loss.backward()
    _, _, ex = rq.factor(_gpu(Xn), 60, 4, rq.GAUSSIAN, passes=2, want_factors=True)
    ref = rq.backward(_gpu(Xn), ex["Rs"], ex["Rp"], _gpu(dQ), _gpu(dR))
    torch.cuda.synchronize()
    assert torch.allclose(X.grad, ref, rtol=0, atol=0)
