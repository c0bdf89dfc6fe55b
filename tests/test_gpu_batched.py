"""Batched factorisation: every instance against its own single call (the
same kernels in the same order: bit for bit) and against the FP64 oracle;
HIP graph capture and replay checked against the eager result."""
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


def _instances(count, seed, m_hi, dtype):
    shapes = synth.batched_shapes(count, seed=seed, m_lo=2000, m_hi=m_hi)
    Xs = [synth.make_x(m, n, 1e-4, seed=100 + i, dtype=dtype) for i, (m, n, k) in enumerate(shapes)]
    return shapes, Xs


@pytest.mark.parametrize("kind,precision,dtype", [(0, 0, np.float64), (1, 2, np.float32),
                                                  (2, 1, np.float32), (3, 2, np.float32),
                                                  (3, 0, np.float64)])
def test_batched_equals_single_calls(rq, kind, precision, dtype):
    import torch
    shapes, Xs = _instances(11, 3, 30000, dtype)
    Xg = [_gpu(X) for X in Xs]
    B = rq.BatchedFactor(Xg, [k for _, _, k in shapes], [7 + i for i in range(len(Xs))],
                         kind=kind, passes=2, precision=precision)
    Qs, Rs = B.run()
    assert B.status() == [0] * len(Xs)
    for i, (m, n, k) in enumerate(shapes):
        Q1, R1 = rq.factor(Xg[i], k, 7 + i, kind, passes=2, precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(Qs[i], Q1) and torch.equal(Rs[i], R1), (i, m, n)


def test_batched_mixed_against_oracle(rq, orc):
    shapes, Xs = _instances(6, 5, 40000, np.float32)
    B = rq.BatchedFactor([_gpu(X) for X in Xs], [k for _, _, k in shapes], list(range(6)),
                         kind=rq.RADEMACHER, passes=2, precision=rq.MIXED)
    Qs, Rs = B.run()
    assert B.status() == [0] * 6
    for i, (m, n, k) in enumerate(shapes):
        X = Xs[i].astype(np.float64)
        Q, R = _np(Qs[i]).astype(np.float64), _np(Rs[i])
        ref = orc.rcholqr(X, k, i, orc.RADEMACHER, passes=2)
        orth = np.linalg.norm(Q.T @ Q - np.eye(n), 2)
        dR = np.linalg.norm(R - ref["R"]) / np.linalg.norm(ref["R"])
        print(f"batched instance {i}: m={m} n={n} orth={orth:.2e} dR={dR:.2e}")
        assert orth <= 1e-6 and dR <= 1e-4


def test_batched_graph_replay(rq):
    """Capture once, replay three times with eager work in between; every
    replay must reproduce the eager batched result bit for bit."""
    import torch
    shapes, Xs = _instances(9, 7, 20000, np.float32)
    Xg = [_gpu(X) for X in Xs]
    ks, seeds = [k for _, _, k in shapes], [3 * i + 1 for i in range(9)]
    eager = rq.BatchedFactor(Xg, ks, seeds, rq.RADEMACHER, 2, rq.MIXED)
    Qe, Re = eager.run()
    torch.cuda.synchronize()
    Qe = [q.clone() for q in Qe]
    Re = [r.clone() for r in Re]
    B = rq.BatchedFactor(Xg, ks, seeds, rq.RADEMACHER, 2, rq.MIXED)
    B.capture()
    other = _gpu(synth.make_x(30000, 40, 1e-3, seed=99, dtype=np.float32))
    for rep in range(3):
        for Q in B.Qs:
            Q.zero_()
        Qs, Rs = B.replay()
        rq.factor(other, 120, 1, rq.RADEMACHER, passes=2, precision=rq.MIXED)  # eager work
        torch.cuda.synchronize()
        for i in range(9):
            assert torch.equal(Qs[i], Qe[i]) and torch.equal(Rs[i], Re[i]), (rep, i)
