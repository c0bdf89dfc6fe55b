"""The persistent batched engine (one launch for a whole batch of FP32
problems, Rademacher sketch): per-problem parity with the FP64 oracle on the
same FP32 values (Algorithms 2 and 3), the batched configuration (512
problems, m in [2000, 200000], n in {16, ..., 128}, k = 3n, sigma 1 -> 1e-4)
with every problem's orthogonality and residual checked on the GPU and a
seeded sample against the oracle, refused problems, bitwise reproducibility,
HIP-graph replays, and the chunk-size tuner with its JSON table."""
import json
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
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
    return rq.fortran(torch.from_numpy(np.asfortranarray(a)).cuda())


def _checks(Xd, Qn, Rn):
    n = Qn.shape[1]
    orth = float(np.linalg.norm(Qn.T @ Qn - np.eye(n), 2))
    res = float(np.max(np.linalg.norm(Xd - Qn @ Rn, axis=0) / np.linalg.norm(Xd, axis=0)))
    return orth, res


def _small_batch(count, seed, m_lo=300, m_hi=30000, sigma=1e-3):
    shapes = synth.batched_shapes(count, seed=seed, m_lo=m_lo, m_hi=m_hi)
    Xs = [synth.make_x(m, n, sigma, seed=seed * 1000 + i, dtype=np.float32)
          for i, (m, n, _) in enumerate(shapes)]
    return shapes, Xs


@pytest.mark.parametrize("passes", [1, 2])
def test_engine_matches_oracle(rq, orc, passes):
    import torch
    shapes, Xs = _small_batch(24, seed=5)
    seeds = [11 + i for i in range(len(Xs))]
    eng = rq.BatchedEngine([_gpu(X) for X in Xs], [k for _, _, k in shapes], seeds,
                           passes=passes, chunk_rows=2048)
    eng.run()
    st = eng.status()
    assert st == [0] * len(Xs), st
    worst = [0.0, 0.0, 0.0]
    for i, (X, (m, n, k)) in enumerate(zip(Xs, shapes)):
        Xd = X.astype(np.float64)
        Qn = eng.Qs[i].cpu().numpy().astype(np.float64)
        Rn = eng.Rs[i].cpu().numpy()
        ref = orc.rcholqr(Xd, k, seeds[i], orc.RADEMACHER, passes=passes)
        assert ref["status"] == 0
        dR = np.linalg.norm(Rn - ref["R"]) / np.linalg.norm(ref["R"])
        orth, res = _checks(Xd, Qn, Rn)
        if passes == 1:
            # Q is well conditioned, not orthonormal: check cond(Q)
            orth = float(np.linalg.cond(Qn))
        worst = [max(worst[0], dR), max(worst[1], orth), max(worst[2], res)]
        assert dR <= 1e-3, (i, m, n, dR)
        assert res <= 1e-5, (i, m, n, res)
        assert (orth <= 1e-5) if passes == 2 else (orth <= 20.0), (i, m, n, orth)
    print(f"engine passes={passes}: worst |dR|/|R| {worst[0]:.2e}, "
          f"{'orth' if passes == 2 else 'cond(Q)'} {worst[1]:.2e}, resid {worst[2]:.2e}")


def test_engine_refuses_bad_problems_and_keeps_the_rest(rq, orc):
    import torch
    shapes, Xs = _small_batch(5, seed=6, m_hi=5000)
    Xg = [_gpu(X) for X in Xs]
    Xbad = _gpu(np.random.default_rng(0).standard_normal((500, 20)).astype(np.float32))
    ks = [k for _, _, k in shapes]
    eng = rq.BatchedEngine(Xg[:2] + [Xbad] + Xg[2:], ks[:2] + [60] + ks[2:], list(range(6)),
                           passes=2, chunk_rows=1024)
    eng.run()
    st = eng.status()
    assert st == [0, 0, rq.BATCH_INVALID, 0, 0, 0], st
    for j, i in enumerate([0, 1, 3, 4, 5]):
        X = Xs[j]
        Qn = eng.Qs[i].cpu().numpy().astype(np.float64)
        orth, res = _checks(X.astype(np.float64), Qn, eng.Rs[i].cpu().numpy())
        assert orth <= 1e-5 and res <= 1e-5


def test_engine_reproducible_and_graph_replays(rq):
    import torch
    shapes, Xs = _small_batch(10, seed=7, m_hi=20000)
    eng = rq.BatchedEngine([_gpu(X) for X in Xs], [k for _, _, k in shapes],
                           list(range(10)), passes=2, chunk_rows=2048)
    eng.run()
    torch.cuda.synchronize()
    Q0 = [q.clone() for q in eng.Qs]
    R0 = [r.clone() for r in eng.Rs]
    eng.run()
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(Q0, eng.Qs))
    assert all(torch.equal(a, b) for a, b in zip(R0, eng.Rs))
    eng.capture()
    for rep in range(3):
        for q in eng.Qs:
            q.zero_()
        for r in eng.Rs:
            r.zero_()
        torch.cuda.synchronize()
        _ = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")
        eng.replay()
        torch.cuda.synchronize()
        assert eng.status() == [0] * len(Xs)
        assert all(torch.equal(a, b) for a, b in zip(Q0, eng.Qs)), rep
        assert all(torch.equal(a, b) for a, b in zip(R0, eng.Rs)), rep


def test_engine_tuner_writes_and_loads_its_table(rq, tmp_path):
    shapes, Xs = _small_batch(6, seed=8, m_hi=20000)
    eng = rq.BatchedEngine([_gpu(X) for X in Xs], [k for _, _, k in shapes],
                           list(range(6)), passes=2, chunk_rows=1024)  # largest workspace
    path = tmp_path / "tune.json"
    try:
        eng.tune(save_path=path)
        table = json.loads(path.read_text())["batched_engine_chunk_rows"]
        maxn = max(n for _, n, _ in shapes)
        tuned = int(table[str(maxn)])
        assert tuned in (1024, 2048, 4096, 8192, 16384)
        rq.init(None)
        assert int(rq.lib().rcholqr_batched_engine_chunk(maxn)) == 8192
        rq.init(path)
        assert int(rq.lib().rcholqr_batched_engine_chunk(maxn)) == tuned
    finally:
        rq.init(None)


@pytest.mark.timeout(900)
def test_engine_batched_configuration(rq, orc):
    """512 problems with the batched configuration's shapes: every status 0,
    every problem's ||Q^T Q - I||_2 and column residual within FP32 bounds
    (on the GPU, FP64 products), a seeded sample (the largest m and one
    problem of each n) against the oracle."""
    import torch
    shapes = synth.batched_shapes(512, seed=0)
    Xs = [synth.make_x_torch(m, n, 1e-4, seed=1000 + i, dtype=torch.float32)
          for i, (m, n, _) in enumerate(shapes)]
    seeds = [1 + i for i in range(len(Xs))]
    eng = rq.BatchedEngine(Xs, [k for _, _, k in shapes], seeds, passes=2)
    eng.run()
    st = eng.status()
    assert st == [0] * len(Xs)
    worst_o = worst_r = 0.0
    for i, X in enumerate(Xs):
        Q = eng.Qs[i].double()
        R = eng.Rs[i]
        n = Q.shape[1]
        orth = torch.linalg.matrix_norm(Q.T @ Q - torch.eye(n, device="cuda", dtype=torch.float64), 2).item()
        Xd = X.double()
        res = (torch.linalg.vector_norm(Xd - Q @ R, dim=0) / torch.linalg.vector_norm(Xd, dim=0)).max().item()
        worst_o, worst_r = max(worst_o, orth), max(worst_r, res)
        assert orth <= 1e-5 and res <= 1e-5, (i, shapes[i], orth, res)
    sample = {int(np.argmax([m for m, _, _ in shapes]))}
    for nv in (16, 32, 64, 96, 128):
        sample.add(next(i for i, (_, n, _) in enumerate(shapes) if n == nv))
    worst_d = 0.0
    for i in sorted(sample):
        m, n, k = shapes[i]
        Xd = np.asfortranarray(Xs[i].double().cpu().numpy())
        ref = orc.rcholqr(Xd, k, seeds[i], orc.RADEMACHER, passes=2)
        dR = np.linalg.norm(eng.Rs[i].cpu().numpy() - ref["R"]) / np.linalg.norm(ref["R"])
        worst_d = max(worst_d, dR)
        assert dR <= 1e-3, (i, shapes[i], dR)
    print(f"engine 512 problems: worst orth {worst_o:.2e}, resid {worst_r:.2e}, "
          f"sample |dR|/|R| {worst_d:.2e}")
