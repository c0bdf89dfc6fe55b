"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.

Tolerances (derivations in the design doc):
* Theta: bit for bit.
* Sketch P: FP64 sums in a different order, |dP| <= 4 m u |Theta||X|.
* Tall solve: both sides are row-wise backward stable (Higham Thm 8.5 as in
  Section 5.1), so they differ by at most ~2 * 1.1 u n cond(R) relative.
* Whole factorisation: eq. (main1) for residuals, eq. (main2)/(main3) for
  the sketched orthogonality, ||Q^T Q - I|| <= 1e-12 and
  max_j ||X_j - (QR)_j|| / ||X_j|| <= 1e-13 in FP64 with two passes.
"""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def rq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_09953_amd as rq
    rq.lib()
    return rq


def _gpu(a, dtype=None):
    import torch
    import paper_2210_09953_amd as rq
    t = torch.from_numpy(np.asfortranarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return rq.fortran(t.to("cuda"))


def _np(t):
    return t.detach().cpu().numpy()


def _colres(X, Q, R):
    return float(np.max(np.linalg.norm(X - Q @ R, axis=0) / np.linalg.norm(X, axis=0)))


# ----------------------------------------------------------------------------- Theta
@pytest.mark.parametrize("kind,k,i0,ni,j0,nj", [
    (0, 150, 0, 150, 0, 4000),
    (0, 601, 0, 601, 999000, 1000),          # odd k, far rows
    (0, 64, 10, 37, (1 << 32) - 20, 64),      # 64-bit row index carry
    (1, 768, 0, 768, 0, 2000),
    (1, 768, 129, 300, 3999000, 1000),
    (2, 600, 0, 600, 0, 3000),
    (2, 1024, 0, 1024, 123456789, 500),
])
def test_theta_bitwise(rq, orc, kind, k, i0, ni, j0, nj):
    g = _np(rq.debug_theta(kind, k, 1, i0, ni, j0, nj))
    c = orc.theta_block(kind, k, 0, 1, i0, ni, j0, nj)
    assert np.array_equal(g.view(np.uint64), c.view(np.uint64))


# ----------------------------------------------------------------------------- sketch
@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("m,n,k", [(3001, 50, 150), (777, 17, 51), (5000, 64, 200)])
def test_sketch_parity_f64(rq, orc, kind, m, n, k):
    X = synth.make_x(m, n, 1e-4, seed=3)
    P = _np(rq.sketch(_gpu(X), k, 11, kind=kind))
    Pr = orc.sketch(kind, X, k, 11)
    th = orc.theta_block(kind, k, m, 11, 0, k, 0, m) * orc.sketch_scale(kind, k)
    bound = 4 * m * U64 * (np.abs(th) @ np.abs(X))
    assert np.all(np.abs(P - Pr) <= bound + 1e-300)


@pytest.mark.parametrize("kind", [0, 2])
def test_sketch_parity_f32_input(rq, orc, kind):
    m, n, k = 4000, 40, 120
    X32 = synth.make_x(m, n, 1e-4, seed=4, dtype=np.float32)
    P = _np(rq.sketch(_gpu(X32), k, 5, kind=kind))
    X = X32.astype(np.float64)
    Pr = orc.sketch(kind, X, k, 5)
    th = orc.theta_block(kind, k, m, 5, 0, k, 0, m) * orc.sketch_scale(kind, k)
    assert np.all(np.abs(P - Pr) <= 4 * m * U64 * (np.abs(th) @ np.abs(X)) + 1e-300)


# ----------------------------------------------------------------------------- solve
@pytest.mark.parametrize("m,n", [(1000, 50), (333, 16), (2049, 200), (130, 1), (700, 256)])
def test_trsm_parity_f64(rq, orc, m, n):
    rng = np.random.default_rng(m + n)
    X = np.asfortranarray(rng.standard_normal((m, n)))
    Rr = np.linalg.qr(rng.standard_normal((3 * n, n)) @ np.diag(np.logspace(0, -5, n)))[1]
    R = np.asfortranarray(Rr * np.sign(np.diag(Rr))[:, None])
    Q = _np(rq.trsm(_gpu(X), _gpu(R)))
    Qr = orc.trsm_rows(X, R)
    cond = np.linalg.cond(R)
    assert np.linalg.norm(Q - Qr) <= 4 * 1.1 * U64 * n * cond * np.linalg.norm(Qr)
    # row-wise backward stability of the GPU solve itself
    assert np.all(np.abs(X - Q @ R) <= 2 * 1.1 * U64 * n * (np.abs(Q) @ np.abs(R)) + 1e-300)


def test_trsm_in_place_f32(rq, orc):
    import torch
    rng = np.random.default_rng(1)
    m, n = 1500, 70
    X = np.asfortranarray(rng.standard_normal((m, n))).astype(np.float32)
    R = np.triu(rng.standard_normal((n, n))) + 8 * np.eye(n)
    Xg = _gpu(X)
    Q = rq.trsm(Xg, _gpu(R), Q=Xg)
    torch.cuda.synchronize()
    Qn = _np(Q).astype(np.float64)
    Qr = orc.trsm_rows(X.astype(np.float64), R)
    assert np.linalg.norm(Qn - Qr) <= 8 * U32 * n * np.linalg.cond(R) * np.linalg.norm(Qr)


@pytest.mark.parametrize("m,n", [(128 * 40 + 37, 96), (128 * 24, 256), (128 * 600 + 5, 128)])
def test_trsm_f32_whole_tiles(rq, orc, m, n):
    """FP32 solve with whole 128-row tiles (staged through LDS) and a ragged
    tail; a padded leading dimension, a misaligned copy (checked kernel) and
    the in-place call give the same bits.  n = 128, 256: persistent
    workgroups; 600 tiles also walk several tiles per workgroup."""
    import torch
    rng = np.random.default_rng(m)
    X = np.asfortranarray(rng.standard_normal((m, n))).astype(np.float32)
    R = np.triu(rng.standard_normal((n, n))) + 8 * np.eye(n)
    Xg = _gpu(X)
    Rg = _gpu(R)
    Q = rq.trsm(Xg, Rg)
    Qr = orc.trsm_rows(X.astype(np.float64), R)
    Qn = _np(Q).astype(np.float64)
    assert np.linalg.norm(Qn - Qr) <= 8 * U32 * n * np.linalg.cond(R) * np.linalg.norm(Qr)
    pad = torch.empty((n, m + 4), dtype=torch.float32, device="cuda")[:, :m].t()
    pad.copy_(Xg)
    mis = torch.empty(m * n + 1, dtype=torch.float32, device="cuda")[1:].view(n, m).t()
    mis.copy_(Xg)
    assert mis.data_ptr() % 16 != 0
    Xi = Xg.clone()
    rq.trsm(Xi, Rg, Q=Xi)
    for other in (rq.trsm(pad, Rg), rq.trsm(mis, Rg), Xi):
        torch.cuda.synchronize()
        assert torch.equal(other, Q)


# ----------------------------------------------------------------------------- factor
def test_config_a_one_pass_parity(rq, orc):
    """m=10000, n=50, k=150, sigma 1 -> 1e-8, Gaussian, FP64, one pass."""
    m, n, k = 10000, 50, 150
    X = synth.make_x(m, n, 1e-8, seed=0)
    Q, R, ex = rq.factor(_gpu(X), k, 1, rq.GAUSSIAN, passes=1, want_s=True, want_factors=True)
    assert rq.status(ex["ws"]) == 0
    Q, R, S = _np(Q), _np(R), _np(ex["S"])
    ref = orc.rcholqr(X, k, 1, orc.GAUSSIAN, passes=1, want_s=True)
    kappa = np.linalg.cond(X / np.linalg.norm(X, axis=0))
    # same Theta => same R up to rounding of P and of the small QR
    assert np.linalg.norm(R - ref["R"]) <= 50 * U64 * n * kappa * np.linalg.norm(ref["R"])
    assert np.linalg.norm(S - ref["S"]) <= 50 * U64 * n * kappa * math.sqrt(n)
    assert np.array_equal(np.tril(R, -1), np.zeros((n, n)))
    assert np.all(np.diag(R) > 0)
    assert _colres(X, Q, R) <= 2.1 * U64 * n                       # eq. (main1)
    th = orc.theta_block(0, k, m, 1, 0, k, 0, m) / math.sqrt(k)
    assert np.linalg.norm(S - th @ Q) <= 6.1 * U64 * n ** 1.5 * kappa   # eq. (main3)
    assert np.linalg.cond(Q) <= 20


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_two_pass_f64_kappa_1e12(rq, orc, kind):
    m, n, k = 20000, 40, 120
    X = synth.make_x(m, n, 1e-12, seed=5)
    Q, R, ex = rq.factor(_gpu(X), k, 9, kind, passes=2, want_factors=True)
    assert rq.status(ex["ws"]) == 0
    Q, R = _np(Q), _np(R)
    assert np.linalg.norm(Q.T @ Q - np.eye(n), 2) <= 1e-12
    assert _colres(X, Q, R) <= 1e-13
    ref = orc.rcholqr(X, k, 9, kind, passes=2)
    # 2-pass R is the unique thin-QR R: GPU and oracle agree to ~u kappa
    assert np.linalg.norm(R - ref["R"]) <= 1e-3 * np.linalg.norm(ref["R"])
    for j in range(n):  # column-wise, relative to each column's own scale
        assert np.linalg.norm(R[:, j] - ref["R"][:, j]) <= 1e-11 * np.linalg.norm(X[:, j]) + \
            U64 * 1e4 * np.linalg.norm(ref["R"][:, j])


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_two_pass_matches_oracle_well_conditioned(rq, orc, kind):
    m, n, k = 5000, 33, 99
    X = synth.make_x(m, n, 1e-3, seed=6)
    Q, R = rq.factor(_gpu(X), k, 3, kind, passes=2)
    ref = orc.rcholqr(X, k, 3, kind, passes=2)
    assert np.linalg.norm(_np(R) - ref["R"]) <= 1e-12 * np.linalg.norm(ref["R"])
    assert np.linalg.norm(_np(Q) - ref["Q"]) <= 1e-12 * np.linalg.norm(ref["Q"])


@pytest.mark.parametrize("kind", [0, 2])
def test_two_pass_f32(rq, orc, kind):
    m, n, k = 30000, 64, 192
    X32 = synth.make_x(m, n, 1e-6, seed=7, dtype=np.float32)
    Q, R, ex = rq.factor(_gpu(X32), k, 2, kind, passes=2, want_factors=True)
    assert rq.status(ex["ws"]) == 0
    Qn = _np(Q).astype(np.float64)
    Rn = _np(R)
    X = X32.astype(np.float64)
    orth = np.linalg.norm(Qn.T @ Qn - np.eye(n), 2)
    res = _colres(X, Qn, Rn)
    ref = orc.rcholqr(X, k, 2, kind, passes=2)
    dR = np.linalg.norm(Rn - ref["R"]) / np.linalg.norm(ref["R"])
    print(f"fp32 2-pass kind={kind}: orth={orth:.2e} resid={res:.2e} dR={dR:.2e}")
    assert orth <= 2e-5
    assert res <= 2e-5
    assert dR <= 1e-4


def test_ragged_shapes_and_single_column(rq, orc):
    for (m, n, k, kind) in [(17, 1, 3, 0), (100, 7, 21, 1), (1031, 129, 387, 0),
                            (80, 64, 64, 1), (900, 255, 765, 2)]:
        X = synth.make_x(m, n, 1e-2, seed=m)
        Q, R = rq.factor(_gpu(X), k, 4, kind, passes=2)
        ref = orc.rcholqr(X, k, 4, kind, passes=2)
        assert ref["status"] == 0
        assert np.linalg.norm(_np(R) - ref["R"]) <= 1e-11 * np.linalg.norm(ref["R"]), (m, n, k)
        assert np.linalg.norm(_np(Q) - ref["Q"]) <= 1e-11 * np.linalg.norm(ref["Q"]), (m, n, k)


def test_status_codes(rq):
    X = synth.make_x(500, 6, 1e-2, seed=6)
    Xz = X.copy()
    Xz[:, 3] = 0.0
    _, _, ex = rq.factor(_gpu(Xz), 18, 1, rq.GAUSSIAN, passes=2, want_factors=True)
    assert rq.status(ex["ws"]) == 1
    Xn = X.copy()
    Xn[7, 2] = np.nan
    _, _, ex = rq.factor(_gpu(Xn), 18, 1, rq.GAUSSIAN, passes=2, want_factors=True)
    assert rq.status(ex["ws"]) == 2
    _, _, ex = rq.factor(_gpu(X), 18, 1, rq.GAUSSIAN, passes=2, want_factors=True)
    assert rq.status(ex["ws"]) == 0


def test_bitwise_deterministic(rq):
    import torch
    X = _gpu(synth.make_x(20000, 48, 1e-6, seed=8))
    for kind in (0, 1, 2):
        a = rq.factor(X, 144, 7, kind, passes=2)
        b = rq.factor(X, 144, 7, kind, passes=2)
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


# ----------------------------------------------------------------------------- mixed
@pytest.mark.parametrize("m,n,k,ramp", [(5000, 64, 192, False), (3333, 200, 600, False),
                                        (1031, 17, 51, False), (20000, 256, 768, False),
                                        (70000, 40, 120, True), (4099, 1, 3, False)])
def test_mixed_sketch_parity(rq, orc, m, n, k, ramp):
    """int8 matrix-core sketch against the FP64 oracle on the same FP32 values.

    The kernel's sums are exact; its only error is quantising each x to a
    multiple of 2^-s with 2^-s <= 2^-20 max_j |x| (the column's maximum over
    the rows seen so far), so |dx| <= 2^-21 max_j |x| and
    ||dP_j|| = ||Theta dx_j|| <= 2 ||dx_j|| <= 2 sqrt(m) 2^-21 max_j |x|
    (the rescaled Rademacher Theta roughly preserves the norm of a vector
    independent of it; 2 leaves room for its fluctuation)."""
    X32 = synth.make_x(m, n, 1e-5, seed=9, dtype=np.float32)
    # wide column scales: the per-column power-of-two scaling must absorb them
    X32 = (X32 * np.float32(10.0) ** np.linspace(-3, 3, n, dtype=np.float32)).astype(np.float32)
    if ramp:  # magnitudes growing down the rows: the column scales change mid-split
        X32 = (X32 * np.float32(10.0) ** np.linspace(-6, 0, m, dtype=np.float32)[:, None])
    X32 = np.asfortranarray(X32.astype(np.float32))
    P = _np(rq.sketch(_gpu(X32), k, 21, kind=rq.RADEMACHER, precision=rq.MIXED))
    X = X32.astype(np.float64)
    Pr = orc.sketch(orc.RADEMACHER, X, k, 21)
    err = np.linalg.norm(P - Pr, axis=0)
    bound = 2.0 * math.sqrt(m) * 2.0 ** -21 * np.abs(X).max(axis=0)
    rel = err / np.linalg.norm(X, axis=0)
    print(f"mixed sketch m={m} n={n}: max ||dP_j||/||X_j|| = {rel.max():.2e}, "
          f"max ||dP_j||/bound_j = {(err / bound).max():.3f}")
    assert np.all(err <= bound)


def test_mixed_status_and_determinism(rq):
    import torch
    X = synth.make_x(3000, 40, 1e-2, seed=6, dtype=np.float32)
    for bad, code in ((np.nan, 2), (np.inf, 2), (-np.inf, 2)):
        Xb = X.copy()
        Xb[1777, 5] = bad
        _, _, ex = rq.factor(_gpu(Xb), 120, 1, rq.RADEMACHER, passes=2, precision=rq.MIXED,
                             want_factors=True)
        assert rq.status(ex["ws"]) == code, bad
    Xz = X.copy()
    Xz[:, 9] = 0.0
    _, _, ex = rq.factor(_gpu(Xz), 120, 1, rq.RADEMACHER, passes=2, precision=rq.MIXED,
                         want_factors=True)
    assert rq.status(ex["ws"]) == 1
    Xg = _gpu(X)
    a = rq.factor(Xg, 120, 4, rq.RADEMACHER, passes=2, precision=rq.MIXED)
    b = rq.factor(Xg, 120, 4, rq.RADEMACHER, passes=2, precision=rq.MIXED)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


@pytest.mark.parametrize("m,n,k,sig", [(50000, 64, 192, 1e-5), (100000, 256, 768, 1e-5)])
def test_mixed_two_pass(rq, orc, m, n, k, sig):
    X32 = synth.make_x(m, n, sig, seed=10, dtype=np.float32)
    Q, R, ex = rq.factor(_gpu(X32), k, 3, rq.RADEMACHER, passes=2, precision=rq.MIXED,
                         want_factors=True)
    assert rq.status(ex["ws"]) == 0
    Qn, Rn = _np(Q).astype(np.float64), _np(R)
    X = X32.astype(np.float64)
    orth = np.linalg.norm(Qn.T @ Qn - np.eye(n), 2)
    res = _colres(X, Qn, Rn)
    ref = orc.rcholqr(X, k, 3, orc.RADEMACHER, passes=2)
    dR = np.linalg.norm(Rn - ref["R"]) / np.linalg.norm(ref["R"])
    dQ = np.linalg.norm(Qn - ref["Q"]) / np.linalg.norm(ref["Q"])
    print(f"mixed 2-pass m={m} n={n}: orth={orth:.2e} resid={res:.2e} dR={dR:.2e} dQ={dQ:.2e}")
    assert orth <= 1e-6
    assert res <= 1e-5
    assert dR <= 1e-4 and dQ <= 1e-3


@pytest.mark.parametrize("precision", ["F32", "MIXED"])
def test_staged_and_checked_paths_agree(rq, orc, precision):
    """m = 40004 (ragged tail), n = 200: the whole-tile solves (staged by
    direct loads) on an aligned X and the checked kernels on a misaligned
    copy give the same bits; both match the oracle."""
    import torch
    m, n, k = 40004, 200, 600
    prec = getattr(rq, precision)
    X32 = synth.make_x(m, n, 1e-5, seed=12, dtype=np.float32)
    Xa = _gpu(X32)
    mis = torch.empty(m * n + 1, dtype=torch.float32, device="cuda")[1:].view(n, m).t()
    mis.copy_(Xa)
    assert mis.data_ptr() % 16 != 0
    Qa, Ra = rq.factor(Xa, k, 6, rq.RADEMACHER, passes=2, precision=prec)
    Qm, Rm = rq.factor(mis, k, 6, rq.RADEMACHER, passes=2, precision=prec)
    torch.cuda.synchronize()
    assert torch.equal(Ra, Rm) and torch.equal(Qa, Qm)
    Qn, Rn = _np(Qa).astype(np.float64), _np(Ra)
    ref = orc.rcholqr(X32.astype(np.float64), k, 6, orc.RADEMACHER, passes=2)
    assert np.linalg.norm(Qn.T @ Qn - np.eye(n), 2) <= 2e-5
    assert _colres(X32.astype(np.float64), Qn, Rn) <= 2e-5
    assert np.linalg.norm(Rn - ref["R"]) <= 1e-4 * np.linalg.norm(ref["R"])


def test_device_copy_is_exact(rq):
    import torch
    src = torch.randint(0, 256, (3 << 20,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    rq.device_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
