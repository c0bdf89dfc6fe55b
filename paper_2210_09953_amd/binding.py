"""ctypes marshalling for librcholqr.so.  No arithmetic of the method here."""
import ctypes
import os

import torch

GAUSSIAN, RADEMACHER, COUNTSKETCH, SRHT = 0, 1, 2, 3
IDENTITY_TESTONLY = 99  # Theta = I, k = m (rcholqr_factor only; a test reduction)
F64, F32, MIXED = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class Problem(ctypes.Structure):
    """Mirror of rcholqr_problem (include/rcholqr.h)."""
    _fields_ = [("X", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("ldx", ctypes.c_int64), ("k", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("Q", ctypes.c_void_p), ("ldq", ctypes.c_int64), ("R", ctypes.c_void_p),
                ("ldr", ctypes.c_int64)]


class LibraryMissing(RuntimeError):
    pass


class RCholQRError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: code {code} ({error_string(code)})")
        self.code = code


def lib_path():
    return os.path.join(_HERE, "librcholqr.so")


def lib():
    """Load librcholqr.so (built in-tree by __graft_entry__.build())."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise LibraryMissing(
            f"{path} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(path)
    i64, u64, i32, sz = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_size_t
    vp, dp = ctypes.c_void_p, ctypes.c_void_p
    L.rcholqr_workspace_bytes.argtypes = [i64, i64, i64, i32, i32, i32]
    L.rcholqr_workspace_bytes.restype = sz
    L.rcholqr_factor.argtypes = [vp, i64, i64, i64, i64, u64, i32, i32, i32, vp, i64, dp,
                                 i64, dp, i64, dp, dp, vp, sz, vp]
    L.rcholqr_factor.restype = i32
    L.rcholqr_status.argtypes = [vp, ctypes.POINTER(i32)]
    L.rcholqr_status.restype = i32
    L.rcholqr_sketch.argtypes = [vp, i64, i64, i64, i64, u64, i32, i32, dp, i64, vp, sz, vp]
    L.rcholqr_sketch.restype = i32
    L.rcholqr_debug_theta.argtypes = [i32, i64, i64, u64, i64, i64, i64, i64, dp, vp]
    L.rcholqr_debug_theta.restype = i32
    L.rcholqr_trsm.argtypes = [vp, i64, i64, i64, dp, i64, i32, vp, i64, vp, sz, vp]
    L.rcholqr_trsm.restype = i32
    L.rcholqr_backward_workspace_bytes.argtypes = [i64, i64, i32]
    L.rcholqr_backward_workspace_bytes.restype = sz
    L.rcholqr_backward.argtypes = [vp, i64, i64, i64, dp, dp, vp, i64, dp, i64, i32, vp, i64,
                                   vp, sz, vp]
    L.rcholqr_backward.restype = i32
    L.rcholqr_batched_workspace_bytes.argtypes = [ctypes.POINTER(Problem), i32, i32, i32, i32]
    L.rcholqr_batched_workspace_bytes.restype = sz
    L.rcholqr_factor_batched.argtypes = [ctypes.POINTER(Problem), i32, i32, i32, i32, vp, sz, vp]
    L.rcholqr_factor_batched.restype = i32
    L.rcholqr_batched_status.argtypes = [ctypes.POINTER(Problem), i32, i32, i32, i32, vp,
                                         ctypes.POINTER(i32)]
    L.rcholqr_batched_status.restype = i32
    L.rcholqr_profile_enable.argtypes = [i32]
    L.rcholqr_profile_enable.restype = i32
    L.rcholqr_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double)]
    L.rcholqr_profile_read.restype = i32
    L.rcholqr_reduced_workspace_bytes.argtypes = [i64, i64, i64, i64, i32, i32]
    L.rcholqr_reduced_workspace_bytes.restype = sz
    L.rcholqr_reduced.argtypes = [vp, i64, i64, i64, i64, i64, u64, i32, i32, dp, i64, dp, i64,
                                  dp, i64, vp, sz, vp]
    L.rcholqr_reduced.restype = i32
    L.rcholqr_col_block_workspace_bytes.argtypes = [i64, i64, i64, i64, i32, i32]
    L.rcholqr_col_block_workspace_bytes.restype = sz
    L.rcholqr_col_block.argtypes = [vp, i64, i64, i64, i64, i64, u64, i32, i32, vp, i64, dp, i64,
                                    dp, i64, vp, sz, vp]
    L.rcholqr_col_block.restype = i32
    L.rcholqr_rr_workspace_bytes.argtypes = [i64, i64, i64, i32, i32, i32]
    L.rcholqr_rr_workspace_bytes.restype = sz
    L.rcholqr_rr.argtypes = [vp, i64, i64, i64, i64, u64, i32, i32, i32, ctypes.c_double,
                             ctypes.c_double, vp, i64,
                             dp, i64, vp, vp, vp, sz, vp]
    L.rcholqr_rr.restype = i32
    L.rcholqr_device_copy.argtypes = [vp, vp, sz, vp]
    L.rcholqr_device_copy.restype = i32
    L.rcholqr_noalloc_max_bytes.argtypes = []
    L.rcholqr_noalloc_max_bytes.restype = sz
    L.rcholqr_factor_noalloc.argtypes = [vp, i64, i64, i64, i64, u64, i32, i32, i32, vp, i64,
                                         dp, i64, vp]
    L.rcholqr_factor_noalloc.restype = i32
    L.rcholqr_noalloc_status.argtypes = [ctypes.POINTER(i32)]
    L.rcholqr_noalloc_status.restype = i32
    L.rcholqr_batched_engine_chunk.argtypes = [i64]
    L.rcholqr_batched_engine_chunk.restype = i64
    L.rcholqr_batched_engine_workspace_bytes.argtypes = [ctypes.POINTER(Problem), i32, i32, i64]
    L.rcholqr_batched_engine_workspace_bytes.restype = sz
    L.rcholqr_factor_batched_engine.argtypes = [vp, i32, i32, i32, i64, vp, sz, vp]
    L.rcholqr_factor_batched_engine.restype = i32
    L.rcholqr_batched_engine_status.argtypes = [i32, vp, ctypes.POINTER(i32)]
    L.rcholqr_batched_engine_status.restype = i32
    L.rcholqr_init.argtypes = [ctypes.c_char_p]
    L.rcholqr_init.restype = i32
    L.rcholqr_batched_engine_tune.argtypes = [ctypes.POINTER(Problem), vp, i32, i32, i32, vp, sz,
                                              ctypes.c_char_p, vp]
    L.rcholqr_batched_engine_tune.restype = i32
    L.rcholqr_error_string.argtypes = [i32]
    L.rcholqr_error_string.restype = ctypes.c_char_p
    _LIB = L
    return L


def error_string(code):
    try:
        return lib().rcholqr_error_string(int(code)).decode()
    except LibraryMissing:
        return "library not built"


def _check(code, what):
    if code != 0:
        raise RCholQRError(code, what)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def empty_fortran(m, n, dtype, device="cuda"):
    return torch.empty_strided((m, n), (1, max(m, 1)), dtype=dtype, device=device)


def fortran(t):
    """Column-major view or copy of a 2-D tensor (stride (1, ld), ld >= m)."""
    m, n = t.shape
    if t.stride(0) == 1 and (n <= 1 or t.stride(1) >= m):
        return t
    out = empty_fortran(m, n, t.dtype, t.device)
    out.copy_(t)
    return out


def _ld(t):
    return max(t.stride(1), t.shape[0], 1) if t.shape[1] > 1 else max(t.shape[0], 1)


def _dtype_for(precision):
    return torch.float64 if precision == F64 else torch.float32


def workspace_bytes(m, n, k, kind, passes, precision):
    return int(lib().rcholqr_workspace_bytes(m, n, k, kind, passes, precision))


def _workspace(m, n, k, kind, passes, precision, ws, device):
    need = workspace_bytes(m, n, k, kind, passes, precision)
    if need == 0:
        raise RCholQRError(-1, "invalid problem size")
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=device)
    if ws.numel() < need:
        raise RCholQRError(-19, "workspace too small")
    return ws


def factor(X, k, seed, kind=GAUSSIAN, passes=2, precision=None, want_s=False,
           want_factors=False, ws=None, Q=None, R=None):
    """Randomized Cholesky QR of a tall X on the GPU (Algorithms 2 and 3).

    Returns (Q, R) or, with want_s / want_factors, (Q, R, extras) where
    extras holds S (k x n), Rs and Rp (the sketch R and the Cholesky factor)
    and the workspace `ws` (its status word is read by status(ws))."""
    if precision is None:
        precision = F64 if X.dtype == torch.float64 else F32
    X = fortran(X)
    m, n = X.shape
    dt = _dtype_for(precision)
    if X.dtype != dt:
        raise TypeError(f"X must be {dt} for precision {precision}")
    dev = X.device
    ws = _workspace(m, n, k, kind, passes, precision, ws, dev)
    if Q is None:
        Q = empty_fortran(m, n, dt, dev)
    if R is None:
        R = empty_fortran(n, n, torch.float64, dev)
    S = empty_fortran(k, n, torch.float64, dev) if want_s else None
    Rs = empty_fortran(n, n, torch.float64, dev) if want_factors else None
    Rp = empty_fortran(n, n, torch.float64, dev) if (want_factors and passes == 2) else None
    code = lib().rcholqr_factor(_ptr(X), m, n, _ld(X), k, int(seed), kind, passes, precision,
                                _ptr(Q), _ld(Q), _ptr(R), _ld(R), _ptr(S), k, _ptr(Rs),
                                _ptr(Rp), _ptr(ws), ws.numel(), _stream())
    _check(code, "rcholqr_factor")
    if want_s or want_factors:
        return Q, R, dict(S=S, Rs=Rs, Rp=Rp, ws=ws)
    return Q, R


def noalloc_max_bytes():
    return int(lib().rcholqr_noalloc_max_bytes())


def factor_noalloc(X, k, seed, kind=GAUSSIAN, passes=2, precision=None, Q=None, R=None):
    """factor() through rcholqr_factor_noalloc: the library's own device
    array is the workspace (no workspace tensor; Q and R are allocated here
    unless given).  Returns (Q, R); noalloc_status() reads the status."""
    if precision is None:
        precision = F64 if X.dtype == torch.float64 else F32
    X = fortran(X)
    m, n = X.shape
    dt = _dtype_for(precision)
    if X.dtype != dt:
        raise TypeError(f"X must be {dt} for precision {precision}")
    if Q is None:
        Q = empty_fortran(m, n, dt, X.device)
    if R is None:
        R = empty_fortran(n, n, torch.float64, X.device)
    code = lib().rcholqr_factor_noalloc(_ptr(X), m, n, _ld(X), k, int(seed), kind, passes,
                                        precision, _ptr(Q), _ld(Q), _ptr(R), _ld(R), _stream())
    _check(code, "rcholqr_factor_noalloc")
    return Q, R


def noalloc_status():
    """Status word of the last completed rcholqr_factor_noalloc call on the
    current device (synchronises)."""
    info = ctypes.c_int(0)
    _check(lib().rcholqr_noalloc_status(ctypes.byref(info)), "rcholqr_noalloc_status")
    return int(info.value)


def reduced(X, k, l, seed, kind=RADEMACHER, precision=None, want_s=False, ws=None):
    """Reduced RCholeskyQR (Algorithm 5): Z = L X R^{-1} (l x n FP64) and R,
    where L is rows k .. k+l-1 of the seeded operator (scaled 1/sqrt(l)).

    Returns (Z, R) or, with want_s, (Z, R, dict(S=S, ws=ws))."""
    if precision is None:
        precision = F64 if X.dtype == torch.float64 else F32
    X = fortran(X)
    m, n = X.shape
    dt = _dtype_for(precision)
    if X.dtype != dt:
        raise TypeError(f"X must be {dt} for precision {precision}")
    need = int(lib().rcholqr_reduced_workspace_bytes(m, n, k, l, kind, precision))
    if need == 0:
        raise RCholQRError(-1, "invalid problem size")
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=X.device)
    if ws.numel() < need:
        raise RCholQRError(-17, "workspace too small")
    Z = empty_fortran(l, n, torch.float64, X.device)
    R = empty_fortran(n, n, torch.float64, X.device)
    S = empty_fortran(k, n, torch.float64, X.device) if want_s else None
    code = lib().rcholqr_reduced(_ptr(X), m, n, _ld(X), k, l, int(seed), kind, precision,
                                 _ptr(Z), _ld(Z), _ptr(R), _ld(R), _ptr(S), k, _ptr(ws),
                                 ws.numel(), _stream())
    _check(code, "rcholqr_reduced")
    if want_s:
        return Z, R, dict(S=S, ws=ws)
    return Z, R


def rr(X, k, seed, kind=GAUSSIAN, precision=None, tau=1e-12, passes=1, f=1.5, ws=None, Q=None,
       R=None):
    """Rank-revealing RCholeskyQR (Algorithm 7; passes=2: RRRCholeskyQR2 with
    one Cholesky QR pass on the kept columns): X[:, piv] ~ Q R with Q (m x r)
    well-conditioned, R (r x n).  The RRQR step is column pivoting followed
    by the strong RRQR swaps with parameter f (f=0: none).  Returns (Q, R,
    piv, r); reading r waits for the stream."""
    if precision is None:
        precision = F64 if X.dtype == torch.float64 else F32
    X = fortran(X)
    m, n = X.shape
    dt = _dtype_for(precision)
    if X.dtype != dt:
        raise TypeError(f"X must be {dt} for precision {precision}")
    need = int(lib().rcholqr_rr_workspace_bytes(m, n, k, kind, precision, passes))
    if need == 0:
        raise RCholQRError(-1, "invalid problem size")
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=X.device)
    if ws.numel() < need:
        raise RCholQRError(-19, "workspace too small")
    if Q is None:
        Q = empty_fortran(m, n, dt, X.device)
    if R is None:
        R = empty_fortran(n, n, torch.float64, X.device)
    piv = torch.empty(n, dtype=torch.int32, device=X.device)
    rank = torch.empty(1, dtype=torch.int32, device=X.device)
    code = lib().rcholqr_rr(_ptr(X), m, n, _ld(X), k, int(seed), kind, precision, int(passes),
                            float(tau), float(f), _ptr(Q), _ld(Q), _ptr(R), _ld(R), _ptr(piv),
                            _ptr(rank), _ptr(ws), ws.numel(), _stream())
    _check(code, "rcholqr_rr")
    r = int(rank.item())
    return Q[:, :r], R[:r, :], piv, r


class ColumnQR:
    """Column-oriented RCholeskyQR (Algorithm 4): append blocks of columns
    one call at a time; Q, S and R grow in buffers sized for n columns.
    After the blocks of j columns, Q[:, :j], S[:, :j] and R[:j, :j] hold the
    factorisation of the columns seen."""

    def __init__(self, m, n, k, seed, kind=GAUSSIAN, precision=F64, device="cuda"):
        self.m, self.n, self.k, self.seed, self.kind, self.precision = m, n, k, seed, kind, precision
        dt = _dtype_for(precision)
        self.Q = empty_fortran(m, n, dt, device)
        self.S = empty_fortran(k, n, torch.float64, device)
        self.R = torch.zeros((n, n), dtype=torch.float64, device=device).t().contiguous().t()
        self.j = 0
        self.ws = None

    def append(self, Xb):
        """Factor the next block X_b (m x b) against the columns so far."""
        Xb = fortran(Xb)
        b = Xb.shape[1]
        if Xb.shape[0] != self.m or self.j + b > self.n:
            raise ValueError("block does not fit")
        need = int(lib().rcholqr_col_block_workspace_bytes(self.m, self.j, b, self.k, self.kind,
                                                           self.precision))
        if need == 0:
            raise RCholQRError(-1, "invalid problem size")
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(need, dtype=torch.uint8, device=Xb.device)
        code = lib().rcholqr_col_block(_ptr(Xb), self.m, self.j, b, _ld(Xb), self.k,
                                       int(self.seed), self.kind, self.precision, _ptr(self.Q),
                                       _ld(self.Q), _ptr(self.S), _ld(self.S), _ptr(self.R),
                                       _ld(self.R), _ptr(self.ws), self.ws.numel(), _stream())
        _check(code, "rcholqr_col_block")
        self.j += b
        return self.Q[:, :self.j], self.R[:self.j, :self.j]


def status(ws):
    """Status word of a workspace after its call finished (synchronises)."""
    info = ctypes.c_int(0)
    _check(lib().rcholqr_status(_ptr(ws), ctypes.byref(info)), "rcholqr_status")
    return int(info.value)


def sketch(X, k, seed, kind=GAUSSIAN, precision=None, ws=None):
    """P = Theta X (k x n FP64, dense kinds scaled by 1/sqrt(k))."""
    if precision is None:
        precision = F64 if X.dtype == torch.float64 else F32
    X = fortran(X)
    m, n = X.shape
    ws = _workspace(m, n, k, kind, 1, precision, ws, X.device)
    P = empty_fortran(k, n, torch.float64, X.device)
    code = lib().rcholqr_sketch(_ptr(X), m, n, _ld(X), k, int(seed), kind, precision, _ptr(P),
                                k, _ptr(ws), ws.numel(), _stream())
    _check(code, "rcholqr_sketch")
    return P


def debug_theta(kind, k, seed, i0, ni, j0, nj, device="cuda", m=1):
    """Raw Theta(i0:i0+ni, j0:j0+nj) as FP64 (test export); m, the rows of X,
    matters for the SRHT only."""
    out = empty_fortran(ni, nj, torch.float64, device)
    code = lib().rcholqr_debug_theta(kind, k, int(m), int(seed), i0, ni, j0, nj, _ptr(out),
                                     _stream())
    _check(code, "rcholqr_debug_theta")
    return out


def trsm(X, R, precision=None, Q=None, ws=None):
    """Q = X R^{-1} by the library's tall triangular solve (R FP64 upper)."""
    if precision is None:
        precision = F64 if X.dtype == torch.float64 else F32
    X = fortran(X)
    R = fortran(R)
    m, n = X.shape
    ws = _workspace(m, n, n, GAUSSIAN, 2, precision, ws, X.device)
    if Q is None:
        Q = empty_fortran(m, n, X.dtype, X.device)
    code = lib().rcholqr_trsm(_ptr(X), m, n, _ld(X), _ptr(R), _ld(R), precision, _ptr(Q),
                              _ld(Q), _ptr(ws), ws.numel(), _stream())
    _check(code, "rcholqr_trsm")
    return Q


PHASES = ("sketch", "small_qr", "solve1", "gram", "cholesky", "solve2")


def profile_enable(on=True):
    """Record HIP events at the phase boundaries of every factor() call."""
    _check(lib().rcholqr_profile_enable(1 if on else 0), "rcholqr_profile_enable")


def profile_read():
    """(calls, {phase: total ms}) since the last read; waits for the events."""
    ms = (ctypes.c_double * len(PHASES))()
    n = lib().rcholqr_profile_read(ms)
    if n < 0:
        raise RCholQRError(n, "rcholqr_profile_read")
    return n, {p: float(ms[i]) for i, p in enumerate(PHASES)}


def device_copy(src, dst):
    """Plain device copy of src into dst (same byte size, 16-byte multiple)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("device_copy: src and dst byte sizes differ")
    _check(lib().rcholqr_device_copy(_ptr(src), _ptr(dst), nb, _stream()),
           "rcholqr_device_copy")


def backward(X, Rs, Rp, dQ, dR=None, precision=None, dX=None, ws=None):
    """dX for the 2-pass factorisation X = Q R given cotangents dQ, dR.

    Q is recomputed from X, Rs, Rp (as saved by factor(..., want_factors=True))
    by the forward kernels; dR may be None (zero)."""
    if precision is None:
        precision = F64 if X.dtype == torch.float64 else F32
    X, dQ = fortran(X), fortran(dQ)
    Rs, Rp = fortran(Rs), fortran(Rp)
    if dR is not None:
        dR = fortran(dR.to(torch.float64))
    m, n = X.shape
    need = int(lib().rcholqr_backward_workspace_bytes(m, n, precision))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=X.device)
    if dX is None:
        dX = empty_fortran(m, n, X.dtype, X.device)
    code = lib().rcholqr_backward(_ptr(X), m, n, _ld(X), _ptr(Rs), _ptr(Rp), _ptr(dQ), _ld(dQ),
                                  _ptr(dR), _ld(dR) if dR is not None else n, precision,
                                  _ptr(dX), _ld(dX), _ptr(ws), ws.numel(), _stream())
    _check(code, "rcholqr_backward")
    return dX


class BatchedFactor:
    """A fixed batch of independent factorisations (one kind, pass count and
    precision), its outputs and its workspace.  run() enqueues one
    rcholqr_factor_batched call on the current stream; capture() records it
    in a HIP graph (torch.cuda.CUDAGraph) and replay() launches that graph."""

    def __init__(self, Xs, ks, seeds, kind=RADEMACHER, passes=2, precision=MIXED):
        self.Xs = [fortran(X) for X in Xs]
        self.kind, self.passes, self.precision = kind, passes, precision
        dt = _dtype_for(precision)
        for X in self.Xs:
            if X.dtype != dt:
                raise TypeError(f"every X must be {dt} for precision {precision}")
        self.Qs = [empty_fortran(X.shape[0], X.shape[1], dt, X.device) for X in self.Xs]
        self.Rs = [empty_fortran(X.shape[1], X.shape[1], torch.float64, X.device)
                   for X in self.Xs]
        n = len(self.Xs)
        self.probs = (Problem * n)()
        for i, (X, Q, R) in enumerate(zip(self.Xs, self.Qs, self.Rs)):
            self.probs[i] = Problem(X.data_ptr(), X.shape[0], X.shape[1], _ld(X), int(ks[i]),
                                    int(seeds[i]), Q.data_ptr(), _ld(Q), R.data_ptr(), _ld(R))
        need = int(lib().rcholqr_batched_workspace_bytes(self.probs, n, kind, passes, precision))
        if need == 0:
            raise RCholQRError(-1, "invalid batched problem")
        self.ws = torch.empty(need, dtype=torch.uint8, device=self.Xs[0].device)
        self.graph = None

    def run(self):
        code = lib().rcholqr_factor_batched(self.probs, len(self.Xs), self.kind, self.passes,
                                            self.precision, _ptr(self.ws), self.ws.numel(),
                                            _stream())
        _check(code, "rcholqr_factor_batched")
        return self.Qs, self.Rs

    def capture(self):
        self.run()                       # creates the stream pool outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
        return self.Qs, self.Rs

    def status(self):
        n = len(self.Xs)
        info = (ctypes.c_int * n)()
        _check(lib().rcholqr_batched_status(self.probs, n, self.kind, self.passes, self.precision,
                                            _ptr(self.ws), info), "rcholqr_batched_status")
        return [int(v) for v in info]


BATCH_INVALID = 3  # engine status of a refused problem


def init(tune_path=None):
    """Load the engine's tuning table (None: built-in defaults)."""
    code = lib().rcholqr_init(None if tune_path is None else str(tune_path).encode())
    _check(code, "rcholqr_init")


class BatchedEngine:
    """A fixed batch of independent FP32 problems factored by the persistent
    batched engine (one launch for the whole batch; Rademacher sketch, 1 or
    2 passes).  The descriptors live on the device (a copy of the host
    array); run() enqueues the engine on the current stream, capture()
    records that in a HIP graph and replay() launches it."""

    def __init__(self, Xs, ks, seeds, passes=2, chunk_rows=0):
        self.Xs = [fortran(X) for X in Xs]
        for X in self.Xs:
            if X.dtype != torch.float32:
                raise TypeError("the batched engine takes FP32 X")
        dev = self.Xs[0].device
        self.passes = passes
        self.Qs = [empty_fortran(X.shape[0], X.shape[1], torch.float32, dev) for X in self.Xs]
        self.Rs = [empty_fortran(X.shape[1], X.shape[1], torch.float64, dev) for X in self.Xs]
        n = len(self.Xs)
        self.probs = (Problem * n)()
        for i, (X, Q, R) in enumerate(zip(self.Xs, self.Qs, self.Rs)):
            self.probs[i] = Problem(X.data_ptr(), X.shape[0], X.shape[1], _ld(X), int(ks[i]),
                                    int(seeds[i]), Q.data_ptr(), _ld(Q), R.data_ptr(), _ld(R))
        raw = bytes(self.probs)
        self.probs_dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
        maxn = max(X.shape[1] for X in self.Xs)
        self.chunk = int(chunk_rows) or int(lib().rcholqr_batched_engine_chunk(maxn))
        need = int(lib().rcholqr_batched_engine_workspace_bytes(self.probs, n, passes, self.chunk))
        if need == 0:
            raise RCholQRError(-1, "invalid batched-engine arguments")
        self.ws = torch.empty(need, dtype=torch.uint8, device=dev)
        self.graph = None

    def run(self):
        code = lib().rcholqr_factor_batched_engine(_ptr(self.probs_dev), len(self.Xs), RADEMACHER,
                                                   self.passes, self.chunk, _ptr(self.ws),
                                                   self.ws.numel(), _stream())
        _check(code, "rcholqr_factor_batched_engine")
        return self.Qs, self.Rs

    def capture(self):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
        return self.Qs, self.Rs

    def status(self):
        """Per-problem status words (synchronises); raises if the engine
        stopped on a bounded wait."""
        n = len(self.Xs)
        info = (ctypes.c_int * n)()
        _check(lib().rcholqr_batched_engine_status(n, _ptr(self.ws), info),
               "rcholqr_batched_engine_status")
        return [int(v) for v in info]

    def tune(self, save_path=None):
        """Time the engine for each chunk size that fits the workspace, keep
        the fastest (written to save_path as JSON when given)."""
        n = len(self.Xs)
        code = lib().rcholqr_batched_engine_tune(self.probs, _ptr(self.probs_dev), n, RADEMACHER,
                                                 self.passes, _ptr(self.ws), self.ws.numel(),
                                                 None if save_path is None else str(save_path).encode(),
                                                 _stream())
        _check(code, "rcholqr_batched_engine_tune")

