"""CPU-side checks of the C ABI: the library loads and exports every symbol
declared in include/rcholqr.h, and argument validation answers without a GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rcholqr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rcholqr_[a-z_]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ["rcholqr_workspace_bytes", "rcholqr_factor", "rcholqr_status",
              "rcholqr_sketch", "rcholqr_debug_theta", "rcholqr_trsm",
              "rcholqr_error_string", "rcholqr_batched_workspace_bytes",
              "rcholqr_factor_batched", "rcholqr_batched_status",
              "rcholqr_backward_workspace_bytes", "rcholqr_backward",
              "rcholqr_reduced_workspace_bytes", "rcholqr_reduced",
              "rcholqr_rr_workspace_bytes", "rcholqr_rr",
              "rcholqr_col_block_workspace_bytes", "rcholqr_col_block"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2210_09953_amd as rq
    L = rq.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_workspace_and_argument_errors_without_gpu():
    import paper_2210_09953_amd as rq
    L = rq.lib()
    assert rq.workspace_bytes(10000, 50, 150, rq.GAUSSIAN, 1, rq.F64) > 0
    assert rq.workspace_bytes(10, 50, 150, rq.GAUSSIAN, 1, rq.F64) == 0   # m < n
    assert rq.workspace_bytes(1000, 50, 40, rq.GAUSSIAN, 1, rq.F64) == 0  # k < n
    assert rq.workspace_bytes(1000, 300, 900, rq.GAUSSIAN, 1, rq.F64) == 0  # n > 256
    vp = ctypes.c_void_p(8)
    # bad n (argument 3), bad k (5), bad passes (8): rejected before any launch
    assert L.rcholqr_factor(vp, 100, 0, 100, 10, 1, 0, 2, 0, vp, 100, vp, 1, None, 1,
                            None, None, vp, 1 << 30, None) == -3
    assert L.rcholqr_factor(vp, 100, 10, 100, 5, 1, 0, 2, 0, vp, 100, vp, 10, None, 1,
                            None, None, vp, 1 << 30, None) == -5
    assert L.rcholqr_factor(vp, 100, 10, 100, 30, 1, 0, 3, 0, vp, 100, vp, 10, None, 1,
                            None, None, vp, 1 << 30, None) == -8
    assert L.rcholqr_factor(vp, 100, 10, 100, 30, 1, 0, 2, 0, vp, 100, vp, 10, None, 1,
                            None, None, vp, 16, None) == -19
    assert rq.error_string(1).startswith("zero diagonal")


def test_batched_argument_errors_without_gpu():
    import paper_2210_09953_amd as rq
    from paper_2210_09953_amd.binding import Problem
    L = rq.lib()
    probs = (Problem * 3)()
    for i in range(3):
        probs[i] = Problem(8, 5000, 32, 5000, 96, i, 8, 5000, 8, 32)
    assert L.rcholqr_batched_workspace_bytes(probs, 3, rq.RADEMACHER, 2, rq.MIXED) > 0
    probs[2].k = 16                                  # k < n in the third instance
    assert L.rcholqr_batched_workspace_bytes(probs, 3, rq.RADEMACHER, 2, rq.MIXED) == 0
    vp = ctypes.c_void_p(8)
    assert L.rcholqr_factor_batched(probs, 3, rq.RADEMACHER, 2, rq.MIXED, vp, 1 << 30,
                                    None) == -2000000 - 2
    assert L.rcholqr_factor_batched(probs, 0, rq.RADEMACHER, 2, rq.MIXED, vp, 1 << 30, None) == -2
    assert L.rcholqr_factor_batched(probs, 3, 7, 2, rq.MIXED, vp, 1 << 30, None) == -3
    probs[2].k = 96
    assert L.rcholqr_factor_batched(probs, 3, rq.RADEMACHER, 2, rq.MIXED, vp, 64, None) == -7


def test_device_copy_argument_errors_without_gpu():
    import paper_2210_09953_amd as rq
    L = rq.lib()
    vp = ctypes.c_void_p
    assert L.rcholqr_device_copy(vp(0), vp(256), 16, None) == -1
    assert L.rcholqr_device_copy(vp(8), vp(256), 16, None) == -1
    assert L.rcholqr_device_copy(vp(256), vp(264), 16, None) == -2
    assert L.rcholqr_device_copy(vp(256), vp(512), 15, None) == -3
    assert L.rcholqr_device_copy(vp(256), vp(512), 0, None) == 0


def test_reduced_argument_errors_without_gpu():
    """Reduced RCholeskyQR: sizes and kinds are checked before any launch."""
    import paper_2210_09953_amd as rq
    L = rq.lib()
    vp = ctypes.c_void_p
    W = L.rcholqr_reduced_workspace_bytes
    assert W(1000, 10, 30, 8, rq.RADEMACHER, rq.F64) > 0
    assert W(1000, 10, 30, 0, rq.RADEMACHER, rq.F64) == 0        # l >= 1
    assert W(1000, 10, 1000, 100, rq.RADEMACHER, rq.F64) == 0    # k + l <= 1024
    assert W(1000, 10, 30, 8, rq.COUNTSKETCH, rq.F64) == 0      # dense kinds only

    def call(X=256, m=1000, n=10, ldx=1000, k=30, l=8, kind=rq.RADEMACHER, prec=rq.F64,
             Z=256, ldz=8, R=256, ldr=10, S=None, lds=30, ws=256, wsb=1 << 30):
        return L.rcholqr_reduced(vp(X), m, n, ldx, k, l, 1, kind, prec, vp(Z), ldz, vp(R), ldr,
                                 vp(S) if S else None, lds, vp(ws), wsb, None)
    assert call(X=0) == -1
    assert call(m=5) == -2
    assert call(ldx=10) == -4
    assert call(k=5) == -5
    assert call(l=0) == -6
    assert call(kind=rq.COUNTSKETCH) == -8
    assert call(kind=rq.GAUSSIAN, prec=rq.MIXED) == -9
    assert call(Z=0) == -10
    assert call(ldz=3) == -11
    assert call(R=0) == -12
    assert call(ldr=4) == -13
    assert call(S=256, lds=10) == -15
    assert call(ws=0) == -16
    assert call(wsb=16) == -17


def test_rr_argument_errors_without_gpu():
    """Rank-revealing RCholeskyQR: sizes, kinds and tau are checked first."""
    import paper_2210_09953_amd as rq
    L = rq.lib()
    vp = ctypes.c_void_p
    assert L.rcholqr_rr_workspace_bytes(1000, 10, 30, rq.GAUSSIAN, rq.F64, 1) > 0
    assert L.rcholqr_rr_workspace_bytes(1000, 10, 30, rq.GAUSSIAN, rq.F64, 2) > \
        L.rcholqr_rr_workspace_bytes(1000, 10, 30, rq.GAUSSIAN, rq.F64, 1)
    assert L.rcholqr_rr_workspace_bytes(1000, 10, 5, rq.GAUSSIAN, rq.F64, 1) == 0
    assert L.rcholqr_rr_workspace_bytes(1000, 10, 30, rq.GAUSSIAN, rq.F64, 3) == 0

    def call(X=256, m=1000, n=10, ldx=1000, k=30, kind=rq.GAUSSIAN, prec=rq.F64, passes=1,
             tau=1e-12, f=1.5, Q=256, ldq=1000, R=256, ldr=10, piv=256, rank=256, ws=256,
             wsb=1 << 30):
        return L.rcholqr_rr(vp(X), m, n, ldx, k, 1, kind, prec, passes, tau, f, vp(Q), ldq,
                            vp(R), ldr, vp(piv), vp(rank), vp(ws), wsb, None)
    assert call(X=0) == -1
    assert call(m=5) == -2
    assert call(n=0) == -3
    assert call(ldx=10) == -4
    assert call(k=5) == -5
    assert call(kind=7) == -7
    assert call(kind=rq.GAUSSIAN, prec=rq.MIXED) == -8
    assert call(passes=0) == -9
    assert call(passes=3) == -9
    assert call(tau=-1.0) == -10
    assert call(tau=float("nan")) == -10
    assert call(f=1.0) == -11
    assert call(f=0.5) == -11
    assert call(f=float("inf")) == -11
    assert call(Q=0) == -12
    assert call(ldq=10) == -13
    assert call(R=0) == -14
    assert call(ldr=3) == -15
    assert call(piv=0) == -16
    assert call(rank=0) == -17
    assert call(ws=0) == -18
    assert call(wsb=16) == -19
    need2 = L.rcholqr_rr_workspace_bytes(1000, 10, 30, rq.GAUSSIAN, rq.F64, 2)
    assert call(passes=2, wsb=need2 - 1) == -19


def test_col_block_argument_errors_without_gpu():
    """Column-oriented RCholeskyQR: sizes and pointers are checked first."""
    import paper_2210_09953_amd as rq
    L = rq.lib()
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    assert L.rcholqr_col_block_workspace_bytes(1000, 10, 6, 48, rq.GAUSSIAN, rq.F64) > 0
    assert L.rcholqr_col_block_workspace_bytes(1000, 10, 6, 12, rq.GAUSSIAN, rq.F64) == 0
    assert L.rcholqr_col_block_workspace_bytes(1000, 250, 7, 1024, rq.GAUSSIAN, rq.F64) == 0

    def call(X=256, m=1000, j0=10, b=6, ldx=1000, k=48, kind=rq.GAUSSIAN, prec=rq.F64, Q=256,
             ldq=1000, S=256, lds=48, R=256, ldr=16, ws=256, wsb=1 << 30):
        return L.rcholqr_col_block(vp(X), m, j0, b, ldx, k, 1, kind, prec, vp(Q), ldq,
                                   ctypes.cast(S, dp), lds, ctypes.cast(R, dp), ldr, vp(ws), wsb,
                                   None)
    assert call(X=0) == -1
    assert call(m=12) == -2
    assert call(j0=-1) == -3
    assert call(b=0) == -4
    assert call(j0=250, b=7) == -4
    assert call(ldx=10) == -5
    assert call(k=12) == -6
    assert call(kind=9) == -8
    assert call(prec=rq.MIXED) == -9
    assert call(Q=0) == -10
    assert call(ldq=10) == -11
    assert call(S=0) == -12
    assert call(lds=10) == -13
    assert call(R=0) == -14
    assert call(ldr=15) == -15
    assert call(ws=0) == -16
    assert call(wsb=16) == -17
