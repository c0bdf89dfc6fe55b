"""rcholqr_factor_noalloc (the entry point for callers that cannot allocate)
against rcholqr_factor: the same launch sequence and kernels on the same
input give the same Q and R, bit for bit, on two calls in a row (the second
smaller, so the library-owned workspace holds the first call's contents when
it starts), for the FP64 and the mixed-precision paths; oversize problems
are refused before any launch."""
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


CASES = [
    # (m, n, k, kind, passes, precision name, sigma_min, x dtype)
    ((60000, 96, 288, 0, 2, "F64", 1e-10, np.float64), (9001, 40, 120, 0, 2, "F64", 1e-6, np.float64)),
    ((120000, 128, 384, 1, 2, "MIXED", 1e-5, np.float32), (20000, 64, 192, 1, 1, "MIXED", 1e-4, np.float32)),
]


@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_matches_factor(rq, first, second):
    import torch
    for (m, n, k, kind, passes, prec, sig, dt) in (first, second):
        precision = getattr(rq, prec)
        need = rq.workspace_bytes(m, n, k, kind, passes, precision)
        assert 0 < need <= rq.noalloc_max_bytes()
        X = _gpu(synth.make_x(m, n, sig, seed=m + n, dtype=dt))
        print(f"noalloc case m={m} n={n} k={k} kind={kind} passes={passes} {prec}", flush=True)
        Q0, R0, ex = rq.factor(X, k, 7, kind, passes=passes, precision=precision,
                               want_factors=True)
        torch.cuda.synchronize()
        st0 = rq.status(ex["ws"])
        Q1, R1 = rq.factor_noalloc(X, k, 7, kind, passes=passes, precision=precision)
        st1 = rq.noalloc_status()
        assert st0 == 0 and st1 == 0
        assert torch.equal(Q0, Q1), "Q differs"
        assert torch.equal(R0, R1), "R differs"


def test_noalloc_refuses_oversize(rq):
    import torch
    m, n, k = 4_000_000, 256, 768
    assert rq.workspace_bytes(m, n, k, rq.GAUSSIAN, 2, rq.F64) > rq.noalloc_max_bytes()
    X = torch.empty(1, device="cuda")  # never read: the size check comes first
    code = rq.lib().rcholqr_factor_noalloc(X.data_ptr(), m, n, m, k, 1, rq.GAUSSIAN, 2,
                                           rq.F64, X.data_ptr(), m, X.data_ptr(), n, None)
    assert code == -3000
