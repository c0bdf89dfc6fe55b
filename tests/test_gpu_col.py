"""GPU parity of column-oriented RCholeskyQR (Algorithm 4), one C-ABI call
per block, against the oracle's col_rcholqr (whose pins tie it to
Algorithm 2 on the whole matrix).  Tolerances as for the one-pass
factorisation: the two sides differ by rounding amplified by cond(R) (the
oracle's least-squares step versus S^T P on the GPU, which agree for
orthonormal S)."""
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


@pytest.mark.parametrize("widths,kind", [((64, 64, 64, 64), 0), ((20, 7, 33, 1), 1),
                                         ((1,) * 12, 0), ((100, 100), 3), ((50,), 2),
                                         ((32, 48, 16), 0)])
def test_col_blocks_f64(rq, orc, widths, kind):
    import torch
    n = sum(widths)
    m, k = 20000, 3 * n
    X = synth.make_x(m, n, 1e-3, seed=14)
    cuts = np.cumsum((0,) + widths)
    blocks = [X[:, a:b] for a, b in zip(cuts[:-1], cuts[1:])]
    cq = rq.ColumnQR(m, n, k, 5, kind, rq.F64)
    prev = None
    for i, Xb in enumerate(blocks):
        cq.append(_gpu(Xb))
        torch.cuda.synchronize()
        if prev is not None:  # the columns already factored stay as they were
            assert np.array_equal(_np(cq.Q[:, :prev.shape[1]]), prev)
        prev = _np(cq.Q[:, :cuts[i + 1]]).copy()
    ref = orc.col_rcholqr(blocks, k, 5, kind)
    Q, S, R = _np(cq.Q), _np(cq.S), _np(cq.R)
    assert np.linalg.norm(R - ref["R"]) <= 1e-11 * np.linalg.norm(ref["R"])
    assert np.linalg.norm(S - ref["S"]) <= 1e-11 * np.linalg.norm(ref["S"])
    assert np.linalg.norm(Q - ref["Q"]) <= 1e-10 * np.linalg.norm(ref["Q"])
    assert np.max(np.linalg.norm(X - Q @ R, axis=0) / np.linalg.norm(X, axis=0)) <= 1e-13


@pytest.mark.parametrize("precision", ["F32", "MIXED"])
def test_col_blocks_f32_and_mixed(rq, orc, precision):
    n, m, k = 128, 30000, 384
    X32 = synth.make_x(m, n, 1e-4, seed=15, dtype=np.float32)
    cq = rq.ColumnQR(m, n, k, 2, rq.RADEMACHER, getattr(rq, precision))
    for a in range(0, n, 32):
        cq.append(_gpu(X32[:, a:a + 32]))
    Q, R = _np(cq.Q).astype(np.float64), _np(cq.R)
    X = X32.astype(np.float64)
    ref = orc.col_rcholqr([X[:, a:a + 32] for a in range(0, n, 32)], k, 2, orc.RADEMACHER)
    res = np.max(np.linalg.norm(X - Q @ R, axis=0) / np.linalg.norm(X, axis=0))
    dR = np.linalg.norm(R - ref["R"]) / np.linalg.norm(ref["R"])
    print(f"col {precision}: resid {res:.2e} dR {dR:.2e} cond(Q) {np.linalg.cond(Q):.2f}")
    assert res <= 1e-5 and dR <= 1e-4
    assert np.linalg.cond(Q) <= 10


def test_col_block_in_place_and_errors(rq, orc):
    """X_b may already sit in Q's next columns (a Krylov step writes it
    there): the same result as from a separate buffer."""
    import torch
    m, n, k = 5000, 40, 120
    X = synth.make_x(m, n, 1e-2, seed=16)
    a = rq.ColumnQR(m, n, k, 9, 0, rq.F64)
    a.append(_gpu(X[:, :24]))
    a.append(_gpu(X[:, 24:]))
    b = rq.ColumnQR(m, n, k, 9, 0, rq.F64)
    b.append(_gpu(X[:, :24]))
    b.Q[:, 24:] = torch.from_numpy(X[:, 24:]).to("cuda")
    b.append(b.Q[:, 24:])
    torch.cuda.synchronize()
    assert torch.equal(a.Q, b.Q) and torch.equal(a.R, b.R)
    with pytest.raises(ValueError):
        a.append(_gpu(X[:, :1]))


@pytest.mark.parametrize("widths", [(240, 16), (96, 32, 128), (20, 7, 33, 68), (64, 64)])
def test_col_blocks_f32_update_pass(rq, orc, widths):
    """The FP32 step 5 reads the solved columns in the same pass that solves
    the new ones: they stay bit for bit as they were, also when j0 is not a
    multiple of 16 (the shared subpanel is solved in place) and when the
    row tiles are shared out to persistent workgroups (m past 256 x 128
    rows), and the result matches the oracle.  The last block is appended a
    second time from inside Q (X_b already in place) with the same bits."""
    import torch
    n = sum(widths)
    m, k = 70000, 3 * n
    X32 = synth.make_x(m, n, 1e-3, seed=17, dtype=np.float32)
    cuts = np.cumsum((0,) + widths)
    cq = rq.ColumnQR(m, n, k, 4, rq.RADEMACHER, rq.F32)
    prev = None
    for i in range(len(widths)):
        cq.append(_gpu(X32[:, cuts[i]:cuts[i + 1]]))
        torch.cuda.synchronize()
        if prev is not None:
            assert np.array_equal(_np(cq.Q[:, :prev.shape[1]]), prev)
        prev = _np(cq.Q[:, :cuts[i + 1]]).copy()
    Q, R = _np(cq.Q).astype(np.float64), _np(cq.R)
    X = X32.astype(np.float64)
    ref = orc.col_rcholqr([X[:, a:b] for a, b in zip(cuts[:-1], cuts[1:])], k, 4, orc.RADEMACHER)
    res = np.max(np.linalg.norm(X - Q @ R, axis=0) / np.linalg.norm(X, axis=0))
    dR = np.linalg.norm(R - ref["R"]) / np.linalg.norm(ref["R"])
    print(f"col f32 {widths}: resid {res:.2e} dR {dR:.2e}")
    assert res <= 1e-5 and dR <= 1e-4
    assert np.linalg.cond(Q) <= 10
    # the last block again, with X_b already in Q's columns
    last = cq.Q.clone()
    cq.j = int(cuts[-2])
    cq.Q[:, cuts[-2]:] = torch.from_numpy(X32[:, cuts[-2]:]).to("cuda")
    cq.append(cq.Q[:, cuts[-2]:])
    torch.cuda.synchronize()
    assert torch.equal(cq.Q, last)
