"""GPU parity of the SRHT sketch (Section 2's subsampled randomized Hadamard
transform) against the oracle.  The oracle transforms whole columns of
length m' with the fast Walsh-Hadamard transform; the library transforms
256-row blocks and adds +-Y[s2] over blocks (srht.hip), and its debug export
forms the entries d_j (-1)^popcount(s_i & j) one by one: three computations
of the same Theta.  Tolerances: Theta bit for bit; P within the FP64 error of
the blocked transform, (16 + blocks + 64) u |Theta||X| (8 butterfly levels,
the sum over a range's blocks, the sum over ranges), for every precision."""
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
    """Mixed precision (FP32 X): at least as accurate as the Rademacher int8
    path's bound, per column ||dP_j|| <= 2 sqrt(m) 2^-21 max|X_j|."""
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
    """k = 1024 (the library's largest) with n = 256: the most samples per
    thread and every column group."""
    m, n, k = 6000, 256, 1024
    X32 = synth.make_x(m, n, 1e-3, seed=5, dtype=np.float32)
    P = _np(rq.sketch(_gpu(X32), k, 8, kind=rq.SRHT, precision=rq.MIXED))
    X = X32.astype(np.float64)
    err = np.linalg.norm(P - orc.sketch(orc.SRHT, X, k, 8), axis=0)
    assert np.all(err <= 2.0 * math.sqrt(m) * 2.0 ** -21 * np.abs(X).max(axis=0))


def _blocked_bound(m, k, Xd):
    """(16 + blocks + 64) u |Theta||X|: every |Theta| entry is 1/sqrt(k)."""
    nb = -(-m // 256)
    return (16 + nb + 64) * U64 * (np.abs(Xd).sum(axis=0) / math.sqrt(k))[None, :]


@pytest.mark.parametrize("m,n,k,ld_extra", [
    (1, 1, 3, 0),                # one row: m' = 1
    (255, 5, 16, 0),             # one ragged block
    (1000, 40, 100, 1),          # odd ld: element loads; three column groups
    (70_000, 17, 300, 0),        # 17 columns, 32 samples per thread
    (300_001, 33, 700, 0),       # 48 samples per thread, ragged last block
    (65_536, 16, 1000, 3),       # 64 samples per thread
    (1_048_653, 16, 768, 0),     # m' = 2^21, many row ranges
])
def test_srht_fast_transform_parity(rq, orc, m, n, k, ld_extra):
    """Every precision against the oracle's FP64 full-length transform,
    within the blocked transform's FP64 bound (far inside 4 m u)."""
    import torch
    X = synth.make_x(m, n, 1e-4, seed=12) if m >= n else np.ones((m, n))
    refs = {np.float64: orc.sketch(orc.SRHT, X, k, 13),
            np.float32: orc.sketch(orc.SRHT, X.astype(np.float32).astype(np.float64), k, 13)}
    for dt, prec in ((np.float64, rq.F64), (np.float32, rq.F32), (np.float32, rq.MIXED)):
        Xh = X.astype(dt)
        buf = torch.zeros((n, m + ld_extra), dtype=torch.float64 if dt == np.float64
                          else torch.float32, device="cuda")
        buf[:, :m] = torch.from_numpy(np.ascontiguousarray(Xh.T)).to("cuda")
        Xg = buf.t()[:m, :]  # column-major, ld = m + ld_extra
        P = _np(rq.sketch(Xg, k, 13, kind=rq.SRHT, precision=prec))
        Xd = Xh.astype(np.float64)
        assert np.all(np.abs(P - refs[dt]) <= _blocked_bound(m, k, Xd) + 1e-300), (dt, prec)


def test_srht_full_size_sampled_columns(rq, orc):
    """The benchmarked launch (m = 4e6, n = 256, k = 768, FP32 X, mixed
    precision: 16 column groups, every row range): four columns of P against
    the oracle's full-length transform of those columns alone (the sketch
    acts on each column separately), within the blocked FP64 bound."""
    import torch
    m, n, k = 4_000_000, 256, 768
    X = synth.make_x_torch(m, n, 1e-5, seed=1, dtype=torch.float32)
    P = _np(rq.sketch(X, k, 7, kind=rq.SRHT, precision=rq.MIXED))
    cols = [0, 17, 128, 255]
    Xc = np.asfortranarray(X[:, cols].double().cpu().numpy())
    del X
    Pr = orc.sketch(orc.SRHT, Xc, k, 7)
    assert np.all(np.abs(P[:, cols] - Pr) <= _blocked_bound(m, k, Xc) + 1e-300)
