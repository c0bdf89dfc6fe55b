"""GPU parity of the SRHT sketch (Section 2's subsampled randomized Hadamard
transform) against the oracle, whose sketch takes the fast Walsh-Hadamard
route while the kernels form the entries d_j (-1)^popcount(s_i & j) on the
fly: two computations of the same Theta.  Tolerances as for the other dense
kinds (test_gpu_parity.py): Theta bit for bit, P within 4 m u |Theta||X|,
the int8 path within its fixed-point rounding bound."""
import math

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


@pytest.mark.parametrize("k,m,i0,ni,j0,nj", [
    (768, 4_000_000, 0, 768, 0, 2000),          # m' = 2^22
    (600, 4_000_000, 129, 300, 3_999_000, 1000),
    (64, 300, 0, 64, 0, 300),                   # ragged m, m' = 512
    (7, 1, 0, 7, 0, 1),                         # m' = 1
    (100, 5_000_000_000, 0, 100, 4_999_999_000, 1000),  # L = 33: 64-bit samples
])
def test_srht_theta_bitwise(rq, orc, k, m, i0, ni, j0, nj):
    g = _np(rq.debug_theta(rq.SRHT, k, 3, i0, ni, j0, nj, m=m))
    c = orc.theta_block(orc.SRHT, k, m, 3, i0, ni, j0, nj)
    assert np.array_equal(g.view(np.uint64), c.view(np.uint64))


@pytest.mark.parametrize("m,n,k", [(3001, 50, 150), (777, 17, 51), (5000, 64, 200)])
def test_srht_sketch_parity_f64_and_f32(rq, orc, m, n, k):
    X = synth.make_x(m, n, 1e-4, seed=3)
    th = orc.theta_block(orc.SRHT, k, m, 11, 0, k, 0, m) / math.sqrt(k)
    for Xin in (X, X.astype(np.float32)):
        Xd = Xin.astype(np.float64)
        P = _np(rq.sketch(_gpu(Xin), k, 11, kind=rq.SRHT))
        Pr = orc.sketch(orc.SRHT, Xd, k, 11)
        assert np.all(np.abs(P - Pr) <= 4 * m * U64 * (np.abs(th) @ np.abs(Xd)) + 1e-300)


@pytest.mark.parametrize("m,n,k", [(5000, 64, 192), (20000, 256, 768), (4099, 1, 3)])
def test_srht_mixed_sketch_parity(rq, orc, m, n, k):
    """int8 matrix cores: exact sums of the quantised X, so per column
    ||dP_j|| <= 2 sqrt(m) 2^-21 max|X_j| (the bound of the Rademacher path)."""
    X32 = synth.make_x(m, n, 1e-5, seed=9, dtype=np.float32)
    X32 = np.asfortranarray((X32 * np.float32(10.0) ** np.linspace(-3, 3, n, dtype=np.float32))
                            .astype(np.float32))
    P = _np(rq.sketch(_gpu(X32), k, 21, kind=rq.SRHT, precision=rq.MIXED))
    X = X32.astype(np.float64)
    Pr = orc.sketch(orc.SRHT, X, k, 21)
    err = np.linalg.norm(P - Pr, axis=0)
    assert np.all(err <= 2.0 * math.sqrt(m) * 2.0 ** -21 * np.abs(X).max(axis=0))


def test_srht_two_pass_f64(rq, orc):
    m, n, k = 20000, 40, 120
    X = synth.make_x(m, n, 1e-3, seed=6)
    Q, R = rq.factor(_gpu(X), k, 3, rq.SRHT, passes=2)
    ref = orc.rcholqr(X, k, 3, orc.SRHT, passes=2)
    assert np.linalg.norm(_np(R) - ref["R"]) <= 1e-12 * np.linalg.norm(ref["R"])
    assert np.linalg.norm(_np(Q) - ref["Q"]) <= 1e-12 * np.linalg.norm(ref["Q"])
    X = synth.make_x(m, n, 1e-12, seed=5)
    Q, R, ex = rq.factor(_gpu(X), k, 9, rq.SRHT, passes=2, want_factors=True)
    assert rq.status(ex["ws"]) == 0
    Q, R = _np(Q), _np(R)
    assert np.linalg.norm(Q.T @ Q - np.eye(n), 2) <= 1e-12
    assert np.max(np.linalg.norm(X - Q @ R, axis=0) / np.linalg.norm(X, axis=0)) <= 1e-13


def test_srht_mixed_two_pass(rq, orc):
    m, n, k = 50000, 64, 192
    X32 = synth.make_x(m, n, 1e-5, seed=10, dtype=np.float32)
    Q, R, ex = rq.factor(_gpu(X32), k, 3, rq.SRHT, passes=2, precision=rq.MIXED,
                         want_factors=True)
    assert rq.status(ex["ws"]) == 0
    Qn, Rn = _np(Q).astype(np.float64), _np(R)
    X = X32.astype(np.float64)
    ref = orc.rcholqr(X, k, 3, orc.SRHT, passes=2)
    orth = np.linalg.norm(Qn.T @ Qn - np.eye(n), 2)
    dR = np.linalg.norm(Rn - ref["R"]) / np.linalg.norm(ref["R"])
    print(f"srht mixed 2-pass: orth={orth:.2e} dR={dR:.2e}")
    assert orth <= 1e-6 and dR <= 1e-4


def test_srht_rank_revealing(rq, orc):
    rng = np.random.default_rng(7)
    m, n, rho, k = 20000, 64, 20, 192
    X = np.asfortranarray((rng.standard_normal((m, rho)) @ rng.standard_normal((rho, n)))
                          * np.logspace(0, 2, n))
    Q, R, piv, r = rq.rr(_gpu(X), k, 5, rq.SRHT, tau=1e-10)
    ref = orc.rr_rcholqr(X, k, 5, orc.SRHT, tau=1e-10)
    assert r == ref["rank"] == rho
    assert np.array_equal(_np(piv)[:r], ref["piv"][:r])
    assert np.linalg.norm(_np(Q) - ref["Q"]) <= 1e-9 * np.linalg.norm(ref["Q"])


def test_srht_mixed_sketch_at_the_largest_k(rq, orc):
    """k = 1024 (the library's largest) with n = 256 runs the main int8 tiles
    with the most Theta row tiles."""
    m, n, k = 6000, 256, 1024
    X32 = synth.make_x(m, n, 1e-3, seed=5, dtype=np.float32)
    P = _np(rq.sketch(_gpu(X32), k, 8, kind=rq.SRHT, precision=rq.MIXED))
    X = X32.astype(np.float64)
    err = np.linalg.norm(P - orc.sketch(orc.SRHT, X, k, 8), axis=0)
    assert np.all(err <= 2.0 * math.sqrt(m) * 2.0 ** -21 * np.abs(X).max(axis=0))
