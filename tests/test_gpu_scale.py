"""GPU parity against the FP64 oracle at the sizes the kernels run at.

These cases reach the code paths that small tests do not: many-stage int8
sketch splits, the FP32 Gram's in-split FP64 flushes (splits of more than
2048 rows), large-m FP64 two-pass runs at kappa = 1e12 (Theorem 5.2,
eq. (main1)-(main3); the experiments of Section 6.1 use m = 1e6), a
Cholesky breakdown reached on the GPU (Algorithm 3 step 3), the adjoint at
1e6 x 128, and inputs built to stress the mixed path's design choices:
columns with one large outlier and heavy-tailed rows (the sketch's
fixed-point scale, Assumption 5.1 / Corollary 2.5), and an R whose 16 x 16
diagonal block is ill conditioned (the FP32 solve's diagonal blocks; the
row-wise backward error of Section 5.1).

Every test prints the measured figures next to its bound.
"""
import ctypes
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


def _gpu(a):
    import torch
    import paper_2210_09953_amd as rq
    return rq.fortran(torch.from_numpy(np.asfortranarray(a)).to("cuda"))


def _np(t):
    return t.detach().cpu().numpy()


def _colres(X, Q, R):
    """max_j ||X_j - (QR)_j|| / ||X_j|| (the residual measure of Section 6.1)."""
    out = 0.0
    for c0 in range(0, X.shape[1], 32):
        c1 = min(X.shape[1], c0 + 32)
        E = X[:, c0:c1] - Q @ R[:, c0:c1]
        out = max(out, float(np.max(np.linalg.norm(E, axis=0) /
                                    np.linalg.norm(X[:, c0:c1], axis=0))))
    return out


def _orth(Q):
    n = Q.shape[1]
    return float(np.linalg.norm(Q.T @ Q - np.eye(n), 2))


def _rowwise_backward_ok(X, Q, R, c):
    """|X - Q R| <= c u n |Q||R| elementwise (Higham Thm 8.5 as in Section 5.1);
    returns the largest ratio of the left side to the bound."""
    n = R.shape[0]
    worst = 0.0
    for r0 in range(0, X.shape[0], 50000):
        r1 = min(X.shape[0], r0 + 50000)
        lhs = np.abs(X[r0:r1] - Q[r0:r1] @ R)
        rhs = n * (np.abs(Q[r0:r1]) @ np.abs(R))
        worst = max(worst, float(np.max(lhs / (c * rhs + 1e-300))))
    return worst


# --------------------------------------------------------------------------- mixed at 1e6 x 256
M1, N1, K1, SEED1 = 1_000_000, 256, 768, 3


@pytest.fixture(scope="module")
def mixed_1m(orc):
    """X (1e6 x 256, sigma 1 -> 1e-5, FP32) and the FP64 oracle's Algorithm 3
    on the same FP32 values (with S and R_s, so P = S R_s is available)."""
    X32 = synth.make_x(M1, N1, 1e-5, seed=21, dtype=np.float32)
    ref = orc.rcholqr(X32.astype(np.float64), K1, SEED1, orc.RADEMACHER, passes=2, want_s=True)
    assert ref["status"] == 0
    return X32, ref


@pytest.mark.timeout(900)
def test_mixed_1m_sketch_against_oracle(rq, mixed_1m):
    """The int8 sketch over many-stage splits: per column, the error is the
    fixed-point rounding of X (|dx| <= 2^-21 of the column's running maximum
    within a row split), so ||dP_j|| <= 2 sqrt(m) 2^-21 max|X_j|."""
    X32, ref = mixed_1m
    P = _np(rq.sketch(_gpu(X32), K1, SEED1, kind=rq.RADEMACHER, precision=rq.MIXED))
    Pr = ref["S"] @ ref["Rs"]
    err = np.linalg.norm(P - Pr, axis=0)
    X = X32.astype(np.float64)
    bound = 2.0 * math.sqrt(M1) * 2.0 ** -21 * np.abs(X).max(axis=0) + \
        1e-14 * np.linalg.norm(Pr, axis=0)
    rel = err / np.linalg.norm(X, axis=0)
    print(f"mixed sketch 1e6x256: max ||dP_j||/||X_j|| = {rel.max():.2e}, "
          f"max ratio to bound {(err / bound).max():.3f}")
    assert np.all(err <= bound)


@pytest.mark.timeout(900)
def test_mixed_1m_two_pass_against_oracle(rq, mixed_1m):
    """The benchmark spec's target: mixed precision at m = 1e6, n = 256, k = 768,
    sigma down to 1e-5: ||Q^T Q - I||_2 <= 1e-6, column residual <= 1e-5,
    R within 1e-4 of the FP64 oracle's (and column by column)."""
    X32, ref = mixed_1m
    Q, R, ex = rq.factor(_gpu(X32), K1, SEED1, rq.RADEMACHER, passes=2, precision=rq.MIXED,
                         want_factors=True)
    assert rq.status(ex["ws"]) == 0
    Qn, Rn = _np(Q).astype(np.float64), _np(R)
    X = X32.astype(np.float64)
    orth = _orth(Qn)
    res = _colres(X, Qn, Rn)
    dR = np.linalg.norm(Rn - ref["R"]) / np.linalg.norm(ref["R"])
    dQ = np.linalg.norm(Qn - ref["Q"]) / np.linalg.norm(ref["Q"])
    dRc = np.max(np.linalg.norm(Rn - ref["R"], axis=0) / np.linalg.norm(ref["R"], axis=0))
    print(f"mixed 1e6x256: orth={orth:.2e} resid={res:.2e} dR={dR:.2e} "
          f"max col dR={dRc:.2e} dQ={dQ:.2e}")
    assert orth <= 1e-6
    assert res <= 1e-5
    assert dR <= 1e-4 and dRc <= 1e-4
    assert dQ <= 1e-3


# --------------------------------------------------------------------------- FP64 at n = 200
@pytest.mark.timeout(900)
@pytest.mark.parametrize("kind", [0, 2])
def test_f64_two_pass_n200_kappa_1e12(rq, orc, kind):
    """Configuration B in FP64 at m = 6e5 (large-m plans: many sketch and
    Gram splits), n = 200, k = 600, sigma 1 -> 1e-12, Gaussian and
    CountSketch: residual <= 1e-13 (eq. (main1)), ||Q^T Q - I|| <= 1e-12,
    R column by column against the oracle's unique thin-QR R."""
    m, n, k = 600_000, 200, 600
    X = synth.make_x(m, n, 1e-12, seed=22)
    Q, R, ex = rq.factor(_gpu(X), k, 5, kind, passes=2, want_factors=True)
    assert rq.status(ex["ws"]) == 0
    Qn, Rn = _np(Q), _np(R)
    orth = _orth(Qn)
    res = _colres(X, Qn, Rn)
    ref = orc.rcholqr(X, k, 5, kind, passes=2)
    assert ref["status"] == 0
    # column j of R: the two sides agree to ~u kappa relative to ||X_j||
    dcol = np.linalg.norm(Rn - ref["R"], axis=0) / np.linalg.norm(X, axis=0)
    print(f"f64 kind={kind} 6e5x200 kappa=1e12: orth={orth:.2e} resid={res:.2e} "
          f"max col ||dR_j||/||X_j|| = {dcol.max():.2e}")
    assert orth <= 1e-12
    assert res <= 1e-13
    assert np.all(dcol <= 1e-3)
    # the well-conditioned leading columns agree to near working precision
    lead = np.linalg.norm(Rn[:, :20] - ref["R"][:, :20]) / np.linalg.norm(ref["R"][:, :20])
    assert lead <= 1e-10


# --------------------------------------------------------------------------- breakdown
def test_cholesky_breakdown_status(rq, orc):
    """Algorithm 3 step 3 fails when Q1 = X R_s^{-1} is not numerically of
    full rank.  Column 17 of X is a vector Theta maps (almost) to zero: two
    rows that CountSketch sends to the same bucket with cancelling signs,
    plus entries of size 2^-700 elsewhere.  R_s[17,17] is then ~2^-700, Q1's
    column 17 is ~1e200 on those two rows, its Gram entries overflow, and
    the pivot of column 17 is Inf - Inf.  Both sides must report 1000 + 17."""
    m, n, k, seed, jb = 200_000, 40, 120, 7, 17
    X = synth.make_x(m, n, 1e-3, seed=3)
    first = {}
    r1 = r2 = None
    for j in range(m):
        h, s = orc.countsketch_hash(k, seed, j)
        if h in first:
            (r1, s1), r2, s2 = first[h], j, s
            break
        first[h] = (j, s)
    z = np.random.default_rng(1).standard_normal(m) * 2.0 ** -700
    z[[r1, r2]] = 0.0
    z[r1], z[r2] = 1.0, -s1 * s2
    X[:, jb] = z
    ref = orc.rcholqr(X, k, seed, orc.COUNTSKETCH, passes=2)
    assert ref["status"] == 1000 + jb
    _, _, ex = rq.factor(_gpu(X), k, seed, rq.COUNTSKETCH, passes=2, want_factors=True)
    st = rq.status(ex["ws"])
    print(f"breakdown: oracle {ref['status']}, GPU {st}")
    assert st == ref["status"]


# --------------------------------------------------------------------------- adjoint 1e6 x 128
@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", [1, 2])
def test_adjoint_config_e(rq, orc, precision):
    """Configuration E: m = 1e6, n = 128, FP32, Rademacher, sigma 1 -> 1e-3:
    the adjoint against the FP64 oracle's closed form, relative error
    <= 1e-3."""
    m, n, k = 1_000_000, 128, 384
    X32 = synth.make_x(m, n, 1e-3, seed=23, dtype=np.float32)
    dQ, dR = synth.make_cotangents(m, n, seed=24)
    dQ32 = dQ.astype(np.float32)
    _, _, ex = rq.factor(_gpu(X32), k, 3, rq.RADEMACHER, passes=2, precision=precision,
                         want_factors=True)
    assert rq.status(ex["ws"]) == 0
    dX = _np(rq.backward(_gpu(X32), ex["Rs"], ex["Rp"], _gpu(dQ32), _gpu(dR),
                         precision=precision)).astype(np.float64)
    ref = orc.rcholqr(X32.astype(np.float64), k, 3, orc.RADEMACHER, passes=2)
    dXr = orc.qr_backward(ref["Q"], ref["R"], dQ32.astype(np.float64), dR)
    err = np.linalg.norm(dX - dXr) / np.linalg.norm(dXr)
    print(f"adjoint 1e6x128 precision={precision}: rel err {err:.2e}")
    assert err <= 1e-3


# --------------------------------------------------------------------------- stress inputs
def _spiky(m, n, sigma, seed):
    """X = U diag(sigma) V^T with one entry per column raised to 1e3 times the
    column's largest magnitude, at a seeded row."""
    X = synth.make_x(m, n, sigma, seed=seed)
    rows = np.random.default_rng(seed).integers(0, m, size=n)
    X[rows, np.arange(n)] = 1e3 * np.abs(X).max(axis=0)
    return X


def _heavy(m, n, sigma, seed):
    """X = diag(w) U diag(sigma) V^T with w_i = |t_3| (Student t, 3 degrees of
    freedom): heavy-tailed row magnitudes."""
    X = synth.make_x(m, n, sigma, seed=seed)
    w = np.abs(np.random.default_rng(seed).standard_t(3, size=m))
    return np.asfortranarray(X * w[:, None])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("shape", ["spiky", "heavy"])
def test_mixed_stress_columns(rq, orc, shape):
    """Mixed precision, 2 passes, m = 1e6, n = 128, k = 384, kappa ~ 1e5, on
    columns with a 1e3x outlier or heavy-tailed rows: the fixed-point sketch
    must still embed (||Q^T Q - I|| <= 1e-6, residual <= 1e-5, R within 1e-4
    of the oracle's on the same FP32 values)."""
    m, n, k = 1_000_000, 128, 384
    X = (_spiky if shape == "spiky" else _heavy)(m, n, 1e-5, 25)
    X32 = np.asfortranarray(X.astype(np.float32))
    Xd = X32.astype(np.float64)
    Q, R, ex = rq.factor(_gpu(X32), k, 4, rq.RADEMACHER, passes=2, precision=rq.MIXED,
                         want_factors=True)
    assert rq.status(ex["ws"]) == 0
    Qn, Rn = _np(Q).astype(np.float64), _np(R)
    ref = orc.rcholqr(Xd, k, 4, orc.RADEMACHER, passes=2)
    assert ref["status"] == 0
    orth = _orth(Qn)
    res = _colres(Xd, Qn, Rn)
    dR = np.linalg.norm(Rn - ref["R"]) / np.linalg.norm(ref["R"])
    print(f"mixed {shape} 1e6x128: orth={orth:.2e} resid={res:.2e} dR={dR:.2e}")
    assert orth <= 1e-6
    assert res <= 1e-5
    assert dR <= 1e-4


def _ill_block_x(m, n, seed, c=0.6):
    """X = U T with Haar U and an upper triangular T that is the identity
    except for a 16 x 16 Kahan block on columns 16..31 (diag s^i, strict upper
    -c s^i, s^2 + c^2 = 1): cond(T_bb) ~ 1e5 and | T_bb^{-1} | | T_bb | large,
    the case where applying a block's inverse loses what substitution keeps."""
    U = synth.make_x(m, n, 1.0, seed=seed)   # sigma = 1: orthonormal columns
    s = math.sqrt(1.0 - c * c)
    K = np.zeros((16, 16))
    for i in range(16):
        K[i, i] = s ** i
        K[i, i + 1:] = -c * s ** i
    T = np.eye(n)
    T[16:32, 16:32] = K
    # a mild grading elsewhere so that the other blocks are not trivial
    T[:, 32:] *= np.logspace(0, -2, n - 32)[None, :]
    return np.asfortranarray(U @ T), K


def test_kahan_block_condition():
    """The construction above reaches the intended diagonal-block conditioning."""
    _, K = _ill_block_x(2000, 48, 1)
    ck = np.linalg.cond(K)
    amp = np.linalg.norm(np.abs(np.linalg.inv(K)) @ np.abs(K), np.inf)
    print(f"Kahan block: cond {ck:.2e}, || |K^-1||K| || = {amp:.2e}")
    assert 1e4 <= ck <= 1e7 and amp >= 1e3


@pytest.mark.parametrize("precision", ["F32", "MIXED"])
def test_ill_conditioned_diagonal_block(rq, orc, precision):
    """FP32 and mixed 2-pass runs whose sketch R has an ill-conditioned 16 x 16
    diagonal block: residual and orthogonality against the FP64 oracle, and the
    row-wise backward error of the GPU's first solve itself."""
    prec = getattr(rq, precision)
    m, n, k = 200_000, 64, 192
    X, _ = _ill_block_x(m, n, 26)
    X32 = np.asfortranarray(X.astype(np.float32))
    Xd = X32.astype(np.float64)
    Q, R, ex = rq.factor(_gpu(X32), k, 6, rq.RADEMACHER, passes=2, precision=prec,
                         want_factors=True)
    assert rq.status(ex["ws"]) == 0
    Qn, Rn = _np(Q).astype(np.float64), _np(R)
    ref = orc.rcholqr(Xd, k, 6, orc.RADEMACHER, passes=2)
    orth = _orth(Qn)
    res = _colres(Xd, Qn, Rn)
    dR = np.linalg.norm(Rn - ref["R"]) / np.linalg.norm(ref["R"])
    # the first solve on its own, with the GPU's R_s
    Rs = _np(ex["Rs"])
    Q1 = _np(rq.trsm(_gpu(X32), ex["Rs"])).astype(np.float64)
    bw = _rowwise_backward_ok(Xd, Q1, Rs, 4 * U32)
    print(f"{precision} Kahan-block 2e5x64: orth={orth:.2e} resid={res:.2e} dR={dR:.2e} "
          f"solve backward error / (4 u32 n |Q||R|) = {bw:.3f}")
    assert orth <= 1e-6 if precision == "MIXED" else orth <= 2e-5
    assert res <= 1e-5
    assert dR <= 1e-4
    assert bw <= 1.0


@pytest.mark.parametrize("m,n", [(128 * 300 + 17, 256), (50000, 96), (4097, 40)])
def test_f32_solve_rowwise_backward_error(rq, orc, m, n):
    """The FP32 tall solve is row-wise backward stable (Section 5.1's
    forward-substitution bound, Higham Thm 8.5, with FP32 unit roundoff):
    |x_i - q_i R| <= 4 u32 n |q_i||R| on every row, for an R with graded
    diagonal blocks."""
    rng = np.random.default_rng(m + n)
    X = np.asfortranarray(rng.standard_normal((m, n))).astype(np.float32)
    Rr = np.linalg.qr(rng.standard_normal((3 * n, n)) @ np.diag(np.logspace(0, -5, n)))[1]
    R = np.asfortranarray(Rr * np.sign(np.diag(Rr))[:, None])
    Q = _np(rq.trsm(_gpu(X), _gpu(R))).astype(np.float64)
    bw = _rowwise_backward_ok(X.astype(np.float64), Q, R, 4 * U32)
    Qr = orc.trsm_rows(X.astype(np.float64), R)
    fwd = np.linalg.norm(Q - Qr) / np.linalg.norm(Qr)
    print(f"f32 solve {m}x{n}: backward error ratio {bw:.3f}, forward {fwd:.2e}")
    assert bw <= 1.0
