"""The test-only embedding Theta = I (k = m) on the GPU: Algorithm 2 then
reduces to Householder QR of X itself, so the GPU's R_s and one-pass Q must
equal LAPACK's thin QR of X with a positive diagonal (the special case of
the method that a textbook routine fixes), and match the oracle's run of
the same reduction.  Two passes leave them unchanged up to rounding."""
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


def _lapack_qr(X):
    Q, R = np.linalg.qr(X)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d, R * d[:, None]


@pytest.mark.parametrize("m,n,passes,dtype", [(700, 100, 1, np.float64), (1024, 256, 1, np.float64),
                                              (333, 40, 2, np.float64), (900, 96, 1, np.float32)])
def test_identity_kind_is_householder_of_x(rq, orc, m, n, passes, dtype):
    import torch
    X = synth.make_x(m, n, 1e-3, seed=m + n, dtype=dtype)
    Xd = X.astype(np.float64)
    prec = rq.F64 if dtype == np.float64 else rq.F32
    Xg = rq.fortran(torch.from_numpy(np.asfortranarray(X)).cuda())
    Q, R, ex = rq.factor(Xg, m, 0, rq.IDENTITY_TESTONLY, passes=passes, precision=prec,
                         want_factors=True)
    torch.cuda.synchronize()
    assert rq.status(ex["ws"]) == 0
    Qn, Rn = Q.cpu().numpy().astype(np.float64), R.cpu().numpy()
    Ql, Rl = _lapack_qr(Xd)
    ref = orc.rcholqr(Xd, m, 0, orc.IDENTITY, passes=passes)
    dRl = np.linalg.norm(Rn - Rl) / np.linalg.norm(Rl)
    dRo = np.linalg.norm(Rn - ref["R"]) / np.linalg.norm(ref["R"])
    dQl = np.linalg.norm(Qn - Ql) / np.linalg.norm(Ql)
    print(f"identity m={m} n={n} passes={passes} {dtype.__name__}: |dR|/|R| vs LAPACK {dRl:.2e}, "
          f"vs oracle {dRo:.2e}; |dQ|/|Q| vs LAPACK {dQl:.2e}")
    # kappa = 1e3: R_s comes from the same FP64 Householder on the same
    # values (FP32 X is promoted exactly), so R agrees to ~u64 kappa; Q is
    # the working-precision solve, whose forward error is ~u kappa sqrt(n)
    # (6e-4 for FP32 at n = 96)
    tol_r = 1e-12
    tol_q = 1e-11 if dtype == np.float64 else 2e-3
    assert dRl <= tol_r and dRo <= tol_r
    assert dQl <= tol_q


def test_identity_kind_argument_rules(rq):
    # k must equal m; the mixed precision has no identity sketch
    assert rq.workspace_bytes(500, 40, 499, rq.IDENTITY_TESTONLY, 1, rq.F64) == 0
    assert rq.workspace_bytes(500, 40, 500, rq.IDENTITY_TESTONLY, 1, rq.MIXED) == 0
    assert rq.workspace_bytes(500, 40, 500, rq.IDENTITY_TESTONLY, 1, rq.F64) > 0


@pytest.mark.parametrize("m,n", [(1024, 200), (777, 33), (256, 256)])
def test_identity_kind_forms_s_as_lapack_q(rq, orc, m, n):
    """With Theta = I the sketch is X itself, so S = (H_1 ... H_n)[I; 0] D of
    Algorithm 2's QR of P is LAPACK's thin Q of X with a positive diagonal R.
    m = 1024 runs the blocked update on four 16-row tiles per wave; n = 200
    and 33 leave a part-filled last panel."""
    import torch
    X = synth.make_x(m, n, 1e-3, seed=3 * m + n)
    Xg = rq.fortran(torch.from_numpy(np.asfortranarray(X)).cuda())
    Q, R, ex = rq.factor(Xg, m, 0, rq.IDENTITY_TESTONLY, passes=1, precision=rq.F64,
                         want_s=True, want_factors=True)
    torch.cuda.synchronize()
    assert rq.status(ex["ws"]) == 0
    S = ex["S"].cpu().numpy()
    Ql, Rl = _lapack_qr(X)
    dS = np.linalg.norm(S - Ql) / np.linalg.norm(Ql)
    orth = np.linalg.norm(S.T @ S - np.eye(n), 2)
    print(f"identity S m={m} n={n}: |dS|/|S| vs LAPACK {dS:.2e}, ||S^T S - I|| {orth:.2e}")
    assert S.shape == (m, n)
    assert dS <= 1e-11            # Q's forward error ~ u kappa sqrt(n), kappa = 1e3
    assert orth <= 1e-13
