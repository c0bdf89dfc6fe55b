"""GPU parity of rank-revealing RCholeskyQR (Algorithm 7) against the oracle.

Compared where the result is unique: the rank, the first r pivots (the
dropped columns are noise-level and their order is not determined), Q's r
columns and R with its columns put back in X's order.  Both sides take the
pivots by the same rule (largest remaining norm, first on ties); the GPU
pivots the R factor of the normalised sketch, which has the sketch's column
norms and inner products, so the decisions agree while the norms are apart.
"""
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


def _gpu(a, dtype=None):
    import torch
    import paper_2210_09953_amd as rq
    t = torch.from_numpy(np.asfortranarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return rq.fortran(t.to("cuda"))


def _np(t):
    return t.detach().cpu().numpy()


def _low_rank(m, n, rho, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((m, rho)) @ rng.standard_normal((rho, n))
    return np.asfortranarray(X * np.logspace(0, 2, n))


def _back_to_x_order(R, piv):
    out = np.zeros_like(R)
    out[:, piv] = R
    return out


@pytest.mark.parametrize("kind,n,rho", [(0, 64, 20), (1, 64, 20), (0, 200, 77), (1, 256, 190)])
def test_rr_low_rank_f64(rq, orc, kind, n, rho):
    """n = 200 and 256 span the four row quarters of the pivoted QR's threads
    (200 with a ragged last quarter)."""
    m, k = 20000, 3 * n
    X = _low_rank(m, n, rho, 7)
    Q, R, piv, r = rq.rr(_gpu(X), k, 5, kind, tau=1e-10)
    ref = orc.rr_rcholqr(X, k, 5, kind, tau=1e-10)
    assert r == ref["rank"] == rho
    piv = _np(piv)
    assert np.array_equal(piv[:r], ref["piv"][:r])
    Q, R = _np(Q), _np(R)
    assert np.linalg.norm(Q - ref["Q"]) <= 1e-9 * np.linalg.norm(ref["Q"])
    Rx, Rx_ref = _back_to_x_order(R, piv), _back_to_x_order(ref["R"], ref["piv"])
    assert np.linalg.norm(Rx - Rx_ref) <= 1e-9 * np.linalg.norm(Rx_ref)
    XP = X[:, piv]
    err = np.linalg.norm(XP - Q @ R, axis=0) / np.linalg.norm(XP, axis=0)
    assert err.max() <= 1e-8
    assert np.linalg.cond(Q) <= 10


@pytest.mark.parametrize("kind", [0, 1])
def test_rr_extreme_column_scales_f64(rq, orc, kind):
    """Columns scaled by 1e170 and 1e-170 (their squares overflow and
    underflow FP64): the column norms take scaled sums, so the result is the
    oracle's (whose norms are scaled too) and, Algorithm 7 normalising by
    D, the same rank and pivots as for the unscaled matrix."""
    m, n, rho, k = 20000, 64, 20, 192
    X0 = _low_rank(m, n, rho, 11)
    sc = np.ones(n)
    sc[0::3], sc[1::3] = 1e170, 1e-170
    X = np.asfortranarray(X0 * sc[None, :])
    Q, R, piv, r = rq.rr(_gpu(X), k, 5, kind, tau=1e-10)
    ref = orc.rr_rcholqr(X, k, 5, kind, tau=1e-10)
    _, _, piv0, r0 = rq.rr(_gpu(X0), k, 5, kind, tau=1e-10)
    assert r == ref["rank"] == int(r0) == rho
    piv = _np(piv)
    assert np.array_equal(piv[:r], ref["piv"][:r])
    assert np.array_equal(piv[:r], _np(piv0)[:r])
    Q, R = _np(Q), _np(R)
    assert np.all(np.isfinite(Q)) and np.all(np.isfinite(R))
    assert np.linalg.norm(Q - ref["Q"]) <= 1e-9 * np.linalg.norm(ref["Q"])
    Rx, Rx_ref = _back_to_x_order(R, piv), _back_to_x_order(ref["R"], ref["piv"])
    cerr = orc.colnorms(Rx - Rx_ref) / orc.colnorms(Rx_ref)  # scaled norms: no Inf
    assert cerr.max() <= 1e-9


def test_rr_full_rank_ill_conditioned_f64(rq, orc):
    """kappa = 1e14: Q stays well-conditioned (the unconditional stability of
    Algorithm 7) and X Pi = Q R to working accuracy on the kept columns."""
    m, n, k = 30000, 40, 120
    X = synth.make_x(m, n, 1e-14, seed=8)
    Q, R, piv, r = rq.rr(_gpu(X), k, 3, 0, tau=1e-15)
    ref = orc.rr_rcholqr(X, k, 3, 0, tau=1e-15)
    assert abs(r - ref["rank"]) <= 1
    Q, R, piv = _np(Q), _np(R), _np(piv)
    assert np.linalg.cond(Q) <= 20
    XP = X[:, piv[:r]]
    err = np.linalg.norm(XP - Q @ R[:, :r], axis=0) / np.linalg.norm(XP, axis=0)
    assert err.max() <= 1e-12


@pytest.mark.parametrize("precision", ["F32", "MIXED"])
def test_rr_low_rank_f32_and_mixed(rq, orc, precision):
    m, n, rho, k = 40000, 64, 24, 192
    X = _low_rank(m, n, rho, 11).astype(np.float32)
    Q, R, piv, r = rq.rr(_gpu(X), k, 9, rq.RADEMACHER, precision=getattr(rq, precision),
                         tau=1e-5)
    ref = orc.rr_rcholqr(X.astype(np.float64), k, 9, orc.RADEMACHER, tau=1e-5)
    assert r == ref["rank"] == rho
    piv = _np(piv)
    assert np.array_equal(piv[:r], ref["piv"][:r])
    Q, R = _np(Q).astype(np.float64), _np(R)
    XP = X.astype(np.float64)[:, piv]
    err = np.linalg.norm(XP - Q @ R, axis=0) / np.linalg.norm(XP, axis=0)
    print(f"rr {precision}: max column error {err.max():.2e} cond(Q) {np.linalg.cond(Q):.2f}")
    assert err.max() <= 1e-4
    assert np.linalg.cond(Q) <= 10


@pytest.mark.parametrize("precision,n,rho", [("F64", 64, 20), ("F64", 200, 200), ("F32", 96, 40),
                                             ("MIXED", 256, 190)])
def test_rr_two_pass(rq, orc, precision, n, rho):
    """RRRCholeskyQR2: the rank and pivots of the single pass, Q orthonormal
    to working accuracy, X Pi = Q R; FP64 against the oracle's second pass."""
    m, k = 20000, 3 * n
    X = _low_rank(m, n, rho, 21)
    kind = 0 if precision == "F64" else rq.RADEMACHER
    tau = 1e-10 if precision == "F64" else 1e-5
    if precision != "F64":
        X = X.astype(np.float32)
    Q, R, piv, r = rq.rr(_gpu(X), k, 6, kind, precision=getattr(rq, precision), tau=tau,
                         passes=2)
    ref = orc.rr_rcholqr2(X.astype(np.float64), k, 6, kind, tau=tau)
    assert r == ref["rank"] == rho
    piv = _np(piv)
    assert np.array_equal(piv[:r], ref["piv"][:r])
    Q, R = _np(Q).astype(np.float64), _np(R)
    orth = np.linalg.norm(Q.T @ Q - np.eye(r), 2)
    XP = X.astype(np.float64)[:, piv]
    err = np.linalg.norm(XP - Q @ R, axis=0) / np.linalg.norm(XP, axis=0)
    print(f"rr2 {precision} n={n}: orth {orth:.2e} max column error {err.max():.2e}")
    if precision == "F64":
        assert orth <= 1e-13
        assert err.max() <= 1e-9
        assert np.linalg.norm(Q - ref["Q"]) <= 1e-9 * np.linalg.norm(ref["Q"])
        Rx, Rx_ref = _back_to_x_order(R, piv), _back_to_x_order(ref["R"], ref["piv"])
        assert np.linalg.norm(Rx - Rx_ref) <= 1e-9 * np.linalg.norm(Rx_ref)
    else:
        assert orth <= 1e-5
        assert err.max() <= 1e-4


def _graded(m, n, seed):
    """U diag(10^(-14 t)) V^T: singular values without a gap, so that column
    pivoting alone leaves a pair for the strong RRQR swaps."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return np.asfortranarray((U * np.logspace(0, -14, n)) @ V.T)


@pytest.mark.parametrize("m,n,seed,kind", [(4000, 64, 1, 0), (4000, 64, 3, 0), (8000, 200, 1, 1)])
def test_rr_strong_swaps_f64(rq, orc, m, n, seed, kind):
    """Inputs where the strong RRQR swaps act (the oracle counts at least
    one): rank, pivots, Q and R as the oracle's; with f = 0 the pivots of
    column pivoting alone."""
    k, tau = 3 * n, 1e-7
    X = _graded(m, n, seed)
    ref = orc.rr_rcholqr(X, k, seed, kind, tau=tau, f=1.5)
    assert ref["swaps"] >= 1
    Q, R, piv, r = rq.rr(_gpu(X), k, seed, kind, tau=tau, f=1.5)
    assert r == ref["rank"]
    piv = _np(piv)
    assert np.array_equal(piv[:r], ref["piv"][:r])
    Q, R = _np(Q), _np(R)
    assert np.linalg.norm(Q - ref["Q"]) <= 1e-7 * np.linalg.norm(ref["Q"])
    Rx, Rx_ref = _back_to_x_order(R, piv), _back_to_x_order(ref["R"], ref["piv"])
    assert np.linalg.norm(Rx - Rx_ref) <= 1e-7 * np.linalg.norm(Rx_ref)
    assert np.linalg.cond(Q) <= 10
    ref0 = orc.rr_rcholqr(X, k, seed, kind, tau=tau, f=0.0)
    _, _, piv0, r0 = rq.rr(_gpu(X), k, seed, kind, tau=tau, f=0.0)
    piv0 = _np(piv0)
    assert r0 == ref0["rank"]
    assert np.array_equal(piv0[:r0], ref0["piv"][:r0])
    assert not np.array_equal(piv0[:r], piv[:r])


def test_rr_degenerate_inputs(rq, orc):
    """A zero X has rank 0 (D = 0, the normalised sketch stays zero); a zero
    column is never kept ahead of a nonzero one; n = 1 keeps its column."""
    import torch
    m, n, k = 3000, 8, 24
    Q, R, piv, r = rq.rr(_gpu(np.zeros((m, n))), k, 1, 0, tau=1e-12)
    assert r == 0 == orc.rr_rcholqr(np.zeros((m, n)), k, 1, 0, tau=1e-12)["rank"]
    assert Q.shape == (m, 0) and R.shape == (0, n)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((m, n))
    X[:, 2] = 0.0
    Q, R, piv, r = rq.rr(_gpu(X), k, 1, 0, tau=1e-12)
    ref = orc.rr_rcholqr(X, k, 1, 0, tau=1e-12)
    assert r == ref["rank"] == n - 1
    piv = _np(piv)
    assert 2 not in piv[:r] and np.array_equal(piv[:r], ref["piv"][:r])
    # n = 1: R = ||Theta x|| (the sketched norm), Q = x / R
    x1 = rng.standard_normal((m, 1))
    Q, R, piv, r = rq.rr(_gpu(x1), 3, 1, 0, tau=1e-12)
    ref = orc.rr_rcholqr(x1, 3, 1, 0, tau=1e-12)
    assert r == 1 and abs(_np(R)[0, 0] - ref["R"][0, 0]) <= 1e-12 * ref["R"][0, 0]
    assert np.linalg.norm(_np(Q) - x1 / ref["R"][0, 0]) <= 1e-12 * np.linalg.norm(_np(Q))
