"""FP64 CPU oracle for randomized Cholesky QR -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke entry and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP product path and never
imports it.  Every routine follows a passage of Balabanov, "Randomized
Cholesky QR factorizations":

* ``sketch``            -- Algorithm 2 step 1, P = Theta X (Section 2 embeddings;
                           the SRHT by its fast Walsh-Hadamard form, ``fwht``)
* ``householder_qr``    -- Algorithm 2 step 2, Householder as in Section 6.1
* ``trsm_rows``         -- Algorithm 2 step 3, row-wise forward substitution
* ``gram``/``cholesky_upper``/``triu_product`` -- Algorithm 3 steps 2-3
* ``rcholqr``           -- Algorithm 2 (passes=1) / Algorithm 3 (passes=2)
* ``col_rcholqr``       -- Algorithm 4 (column-oriented RCholeskyQR, Section 3.2)
* ``reduced_rcholqr``   -- Algorithm 5 (Reduced RCholeskyQR, Section 3.3)
* ``qrcp``/``strong_rrqr``/``rr_rcholqr`` -- Algorithm 7 (rank-revealing
                           RCholeskyQR, Section 4); its RRQR step is QR with
                           column pivoting and the strong RRQR swaps
* ``rr_rcholqr2``       -- RRRCholeskyQR2 (Section 4): Algorithm 7 and one
                           Cholesky QR pass (Algorithm 3 steps 2-4)
* ``qr_backward``       -- reverse-mode derivative of the positive-diagonal
                           thin QR (not in the paper; standard identity)

Parity pins for each routine are in tests/test_oracle_pins.py.  Arrays are
numpy float64 in Fortran (column-major) order, like the C-ABI of the product.
"""
import ctypes
import os

import numpy as np

from . import build as _build

GAUSSIAN, RADEMACHER, COUNTSKETCH, SRHT, IDENTITY = 0, 1, 2, 3, 99

SRHT_TAG_SIGNS, SRHT_TAG_ROWS = 0x53524844, 0x53524853  # "SRHD", "SRHS"

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or (
                os.path.getmtime(path) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = ctypes.CDLL(path)
        i64, u64, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
        dp = ctypes.POINTER(ctypes.c_double)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_threads.restype = i32
        L.orc_ln.argtypes = [ctypes.c_double]
        L.orc_ln.restype = ctypes.c_double
        L.orc_sincos2pi_dyadic.argtypes = [u64, dp, dp]
        L.orc_theta_block.argtypes = [i32, i64, i64, u64, i64, i64, i64, i64, dp]
        L.orc_countsketch_hash.argtypes = [i64, u64, i64,
                                           ctypes.POINTER(i64), dp]
        L.orc_sketch_scale.argtypes = [i32, i64]
        L.orc_sketch_scale.restype = ctypes.c_double
        L.orc_sketch.argtypes = [i32, i64, i64, i64, u64, dp, i64, dp, i64]
        L.orc_householder_qr.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
        L.orc_householder_qr.restype = i32
        L.orc_trsm_rows.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
        L.orc_gram.argtypes = [i64, i64, dp, i64, dp, i64]
        L.orc_cholesky_upper.argtypes = [i64, dp, i64, dp, i64]
        L.orc_cholesky_upper.restype = i32
        L.orc_triu_product.argtypes = [i64, dp, i64, dp, i64, dp, i64]
        L.orc_rcholqr.argtypes = [i32, i32, i64, i64, i64, u64, dp, i64, dp,
                                  i64, dp, i64, dp, i64, dp, dp]
        L.orc_rcholqr.restype = i32
        L.orc_qr_backward.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, dp,
                                      i64, dp, i64]
        _lib = L
    return _lib


def _f64(a):
    a = np.asarray(a, dtype=np.float64)
    return np.asfortranarray(a)


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def philox4x32_10(counter, key):
    """One Philox4x32-10 block (Salmon et al. SC'11) -> 4 uint32 words."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xffffffff for x in counter])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xffffffff for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(o[i]) for i in range(4)]


def threads():
    """Threads the oracle's parallel loops use."""
    return int(lib().orc_threads())


def ln(x: float) -> float:
    return lib().orc_ln(float(x))


def sincos2pi_dyadic(b: int):
    """(sin, cos) of 2*pi*b*2^-53 for integer b in [0, 2^53)."""
    s, c = ctypes.c_double(), ctypes.c_double()
    lib().orc_sincos2pi_dyadic(int(b), ctypes.byref(s), ctypes.byref(c))
    return s.value, c.value


def srht_log2(m):
    """L with m' = 2^L the least power of two >= m."""
    L = 0
    while (1 << L) < m:
        L += 1
    return L


def srht_signs(seed, m, j0=0):
    """The diagonal D of the SRHT for rows j0 .. m-1: d_j = -1 where bit
    (8e + t) of word q of Philox((blk, 0, SRHD), seed) is set, j = 128 blk +
    32 q + 4 t + e."""
    d = np.ones(m - j0)
    for blk in range(j0 // 128, (m + 127) // 128):
        w = philox4x32_10((blk & 0xffffffff, blk >> 32, 0, SRHT_TAG_SIGNS),
                          (seed & 0xffffffff, seed >> 32))
        for r in range(128):
            j = 128 * blk + r
            if j0 <= j < m:
                q, t, e = r >> 5, (r & 31) >> 2, r & 3
                if (w[q] >> (8 * e + t)) & 1:
                    d[j - j0] = -1.0
    return d


def _parity(a):
    """Parity of the set bits of each non-negative int64 (XOR folding)."""
    a = np.array(a, dtype=np.int64, copy=True)
    for sh in (32, 16, 8, 4, 2, 1):
        a ^= a >> sh
    return a & 1


def srht_rows(seed, k, m):
    """The k sampled rows of the SRHT, uniform on [0, m') and independent:
    the top L bits of the 64-bit word (w1 w0) of Philox((i, 0, SRHS), seed)."""
    L = srht_log2(m)
    s = np.zeros(k, dtype=np.int64)
    for i in range(k):
        w = philox4x32_10((i, 0, 0, SRHT_TAG_ROWS), (seed & 0xffffffff, seed >> 32))
        x = (w[1] << 32) | w[0]
        s[i] = 0 if L == 0 else x >> (64 - L)
    return s


def fwht(Y):
    """Unnormalised fast Walsh-Hadamard transform along axis 0 (length a power
    of two): Y <- H Y with H the Sylvester-Hadamard matrix of +-1."""
    Y = np.array(Y, dtype=np.float64, copy=True)
    h, mp = 1, Y.shape[0]
    while h < mp:
        Y = Y.reshape(mp // (2 * h), 2, h, -1)
        a, b = Y[:, 0].copy(), Y[:, 1].copy()
        Y[:, 0], Y[:, 1] = a + b, a - b
        Y = Y.reshape(mp, -1)
        h *= 2
    return Y


def theta_block(kind, k, m, seed, i0, ni, j0, nj):
    """Raw Theta(i0:i0+ni, j0:j0+nj): z for Gaussian, +-1 for Rademacher,
    s(j) at row h(j) for CountSketch, d_j (-1)^popcount(s_i & j) for the
    SRHT (no 1/sqrt(k) scaling)."""
    if kind == SRHT:
        s = srht_rows(seed, k, m)[i0:i0 + ni]
        d = srht_signs(seed, j0 + nj, j0)
        j = np.arange(j0, j0 + nj, dtype=np.int64)
        par = _parity(s[:, None] & j[None, :]).astype(np.float64)
        return np.asfortranarray((1.0 - 2.0 * par) * d[None, :])
    out = np.zeros((ni, nj), dtype=np.float64, order="F")
    lib().orc_theta_block(kind, k, m, seed, i0, ni, j0, nj, _ptr(out))
    return out


def countsketch_hash(k, seed, j):
    h, s = ctypes.c_int64(), ctypes.c_double()
    lib().orc_countsketch_hash(k, seed, j, ctypes.byref(h), ctypes.byref(s))
    return h.value, s.value


def sketch_scale(kind, k):
    if kind == SRHT:
        return 1.0 / np.sqrt(k)
    return lib().orc_sketch_scale(kind, k)


def sketch(kind, X, k, seed):
    """P = Theta X (Algorithm 2 step 1).  The SRHT takes its fast form (the
    n m log m cost the paper counts): signs, the Walsh-Hadamard transform of
    the rows padded to m' = 2^L, then the sampled rows scaled by 1/sqrt(k)."""
    X = _f64(X)
    m, n = X.shape
    if kind == SRHT:
        Y = np.zeros((1 << srht_log2(m), n))
        Y[:m] = srht_signs(seed, m)[:, None] * X
        Y = fwht(Y)
        return np.asfortranarray(Y[srht_rows(seed, k, m)] / np.sqrt(k))
    P = np.zeros((k, n), dtype=np.float64, order="F")
    lib().orc_sketch(kind, m, n, k, seed, _ptr(X), max(m, 1), _ptr(P), k)
    return P


def householder_qr(P, want_s=True):
    P = _f64(P)
    k, n = P.shape
    R = np.zeros((n, n), order="F")
    S = np.zeros((k, n), order="F") if want_s else None
    st = lib().orc_householder_qr(k, n, _ptr(P), k, _ptr(R), n, _ptr(S), k)
    return R, S, st


def trsm_rows(X, R):
    X, R = _f64(X), _f64(R)
    m, n = X.shape
    Q = np.zeros((m, n), order="F")
    lib().orc_trsm_rows(m, n, _ptr(X), max(m, 1), _ptr(R), n, _ptr(Q), max(m, 1))
    return Q


def gram(Q):
    Q = _f64(Q)
    m, n = Q.shape
    G = np.zeros((n, n), order="F")
    lib().orc_gram(m, n, _ptr(Q), max(m, 1), _ptr(G), n)
    return G


def cholesky_upper(G):
    G = _f64(G)
    n = G.shape[0]
    Rp = np.zeros((n, n), order="F")
    st = lib().orc_cholesky_upper(n, _ptr(G), n, _ptr(Rp), n)
    return Rp, st


def triu_product(A, B):
    A, B = _f64(A), _f64(B)
    n = A.shape[0]
    C = np.zeros((n, n), order="F")
    lib().orc_triu_product(n, _ptr(A), n, _ptr(B), n, _ptr(C), n)
    return C


def rcholqr(X, k, seed, kind=GAUSSIAN, passes=2, want_s=False):
    """Algorithm 2 (passes=1) or Algorithm 3 (passes=2).

    Returns dict(Q, R, Rs, Rp, S, status).  FP32 inputs are promoted to
    FP64 exactly; the oracle always computes in FP64.  The SRHT runs the
    same steps from the routines above (sketch, Householder, row solve,
    Gram, Cholesky, product)."""
    X = _f64(X)
    m, n = X.shape
    if kind == SRHT:
        Rs, S, st = householder_qr(sketch(SRHT, X, k, seed), want_s)
        Q = trsm_rows(X, Rs)
        out = dict(Q=Q, R=Rs, Rs=Rs, Rp=None, S=S, status=int(st))
        if passes == 2:
            Rp, st2 = cholesky_upper(gram(Q))
            out.update(Q=trsm_rows(Q, Rp), R=triu_product(Rp, Rs), Rp=Rp,
                       status=int(st) or int(st2))
        return out
    Q = np.zeros((m, n), order="F")
    R = np.zeros((n, n), order="F")
    Rs = np.zeros((n, n), order="F")
    Rp = np.zeros((n, n), order="F")
    S = np.zeros((k, n), order="F") if want_s else None
    st = lib().orc_rcholqr(kind, passes, m, n, k, seed, _ptr(X), max(m, 1),
                           _ptr(Q), max(m, 1), _ptr(R), n, _ptr(S), k,
                           _ptr(Rs), _ptr(Rp))
    return dict(Q=Q, R=R, Rs=Rs, Rp=Rp if passes == 2 else None, S=S,
                status=int(st))


def col_rcholqr(blocks, k, seed, kind=GAUSSIAN):
    """Algorithm 4 (column-oriented RCholeskyQR, Section 3.2) over the column
    blocks X_(1), ..., X_(p) of X (given up front here; in an application each
    comes from the Q of the previous ones): P_i = Theta X_i; R_{1:i-1,i} the
    least-squares solution of S_{1:i-1} R = P_i (numpy's lstsq); [S_i, R_ii]
    the Householder QR of P_i - S_{1:i-1} R_{1:i-1,i}; Q_i = (X_i -
    Q_{1:i-1} R_{1:i-1,i}) R_ii^{-1} by the row-wise forward substitution.
    Returns dict(Q, S, R)."""
    blocks = [_f64(b) for b in blocks]
    m = blocks[0].shape[0]
    n = sum(b.shape[1] for b in blocks)
    Q = np.zeros((m, n), order="F")
    S = np.zeros((k, n), order="F")
    R = np.zeros((n, n), order="F")
    j0 = 0
    for Xi in blocks:
        b = Xi.shape[1]
        Pi = sketch(kind, Xi, k, seed)
        if j0:
            Rc = np.linalg.lstsq(S[:, :j0], Pi, rcond=None)[0]
            R[:j0, j0:j0 + b] = Rc
            W = Pi - S[:, :j0] @ Rc
            Y = Xi - Q[:, :j0] @ Rc
        else:
            W, Y = Pi, Xi
        Rii, Si, _ = householder_qr(np.asfortranarray(W))
        S[:, j0:j0 + b] = Si
        R[j0:j0 + b, j0:j0 + b] = Rii
        Q[:, j0:j0 + b] = trsm_rows(np.asfortranarray(Y), Rii)
        j0 += b
    return dict(Q=Q, S=S, R=R)


def extractor(kind, k, l, m, seed):
    """L for the reduced variant: rows k .. k+l-1 of the seeded operator
    (the rows after Theta's), scaled like an l-row embedding (1/sqrt(l)).
    Dense kinds only (a CountSketch row set is not a CountSketch)."""
    if kind not in (GAUSSIAN, RADEMACHER):
        raise ValueError("extractor rows need a dense sketch kind")
    return theta_block(kind, k + l, m, seed, k, l, 0, m) * sketch_scale(kind, l)


def reduced_rcholqr(X, k, l, seed, kind=RADEMACHER, want_s=False):
    """Algorithm 5: P = Theta X and Y = L X (step 1), [S, R] = QR(P)
    (step 2, Householder with positive diagonal), Z = Y R^{-1} (step 3,
    row-wise forward substitution).  Returns dict(Z, R, S, P, Y, status)."""
    X = _f64(X)
    m, n = X.shape
    P = sketch(kind, X, k, seed)
    Y = np.asfortranarray(extractor(kind, k, l, m, seed) @ X)
    R, S, st = householder_qr(P, want_s=want_s)
    Z = trsm_rows(Y, R) if st == 0 else None
    return dict(Z=Z, R=R, S=S, P=P, Y=Y, status=int(st))


def qrcp(A):
    """Householder QR with column pivoting (Businger-Golub): at step j the
    remaining column of largest 2-norm over rows j.. (recomputed, first one
    on ties) is swapped in, then reflected.  Returns (R, piv) with A[:, piv]
    = Q R and a positive diagonal of R (rows of R and columns of Q flipped)."""
    W = np.array(_f64(A), dtype=np.float64, order="F", copy=True)
    k, n = W.shape
    piv = np.arange(n)
    for j in range(min(k, n)):
        norms = np.sqrt(np.sum(W[j:, j:] ** 2, axis=0))
        p = j + int(np.argmax(norms))
        if p != j:
            W[:, [j, p]] = W[:, [p, j]]
            piv[[j, p]] = piv[[p, j]]
        x = W[j:, j].copy()
        nrm = np.linalg.norm(x)
        if nrm == 0.0:
            continue
        alpha = -nrm if x[0] >= 0 else nrm
        v = x.copy()
        v[0] -= alpha
        beta = 2.0 / (v @ v)
        W[j:, j:] -= beta * np.outer(v, v @ W[j:, j:])
        W[j, j] = alpha
        W[j + 1:, j] = 0.0
    R = np.triu(W[:n, :n]) if k >= n else np.triu(W)
    sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
    return np.asfortranarray(R * sgn[:, None]), piv


def rr_rank(R, tau):
    """Step 3 of Algorithm 7: the least r with ||R[r:, r:]||_F <= tau ||R||_2."""
    n = R.shape[0]
    s2 = np.linalg.norm(R, 2)
    for r in range(n + 1):
        if np.linalg.norm(R[r:, r:], "fro") <= tau * s2:
            return r
    return n


def strong_rrqr(R, k, f=1.5, max_swaps=None):
    """Strong RRQR (Gu and Eisenstat, 1996, the method Section 4 names for the
    RRQR step, with f = 1.5 in the experiments) applied to a QR factor R
    (n x n, upper triangular) for a fixed k: while some pair (i, j) has
    rho_ij^2 = (R11^{-1} R12)_ij^2 + (||R22 e_j|| ||e_i^T R11^{-1}||)^2 > f^2,
    columns i and k + j trade places and R is triangularised again; each such
    swap raises |det R11| by the factor rho_ij > f.  The largest rho_ij
    (first in row-major order on ties) is taken each time.  Returns (R with a
    positive diagonal, perm, swaps): the input's columns perm, factored."""
    R = np.array(_f64(R), dtype=np.float64, order="F", copy=True)
    n = R.shape[0]
    perm = np.arange(n)
    cap = 4 * n if max_swaps is None else max_swaps
    swaps = 0
    while 0 < k < n and swaps < cap:
        Rinv = np.linalg.solve(R[:k, :k], np.eye(k))
        A = Rinv @ R[:k, k:]
        w = np.linalg.norm(Rinv, axis=1)       # 1 / omega_i
        g = np.linalg.norm(R[k:, k:], axis=0)  # gamma_j
        rho2 = A ** 2 + np.outer(w, g) ** 2
        i, j = np.unravel_index(int(np.argmax(rho2)), rho2.shape)
        if not rho2[i, j] > f * f:
            break
        R[:, [i, k + j]] = R[:, [k + j, i]]
        perm[[i, k + j]] = perm[[k + j, i]]
        R = np.linalg.qr(R, mode="r")
        R = np.asfortranarray(R * np.where(np.diag(R) < 0, -1.0, 1.0)[:, None])
        swaps += 1
    return R, perm, swaps


def colnorms(X):
    """Column 2-norms ||X_j||, the D of Algorithm 7.  Each column is divided
    by its largest magnitude before squaring, so that no square overflows or
    underflows (a plain sum of squares is Inf for entries near 1e170 and 0
    near 1e-170); a zero column has norm 0."""
    X = _f64(X)
    a = np.abs(X).max(axis=0) if X.shape[0] else np.zeros(X.shape[1])
    s = np.where(a > 0, a, 1.0)
    return s * np.sqrt(((X / s[None, :]) ** 2).sum(axis=0))


def rr_rcholqr(X, k, seed, kind=GAUSSIAN, tau=1e-12, f=1.5):
    """Algorithm 7 on the column-normalised X (Section 4): D = column norms,
    P = (Theta X) D^{-1}, [R, Pi] = RRQR(P), rank r, Q = (X Pi_{1:r})
    (R_{1:r,1:r} (Pi^T D Pi)_{1:r})^{-1} and R <- R_{1:r,:} Pi^T D Pi.  The
    RRQR is column-pivoted Householder followed, when f > 0, by the strong
    RRQR swaps for k = the rank that the rule gives on the pivoted R; the
    rule is then applied again.  Returns dict(Q, R, piv, rank, Rn, swaps)
    (Rn: the R of the normalised sketch)."""
    X = _f64(X)
    m, n = X.shape
    d = colnorms(X)
    P = sketch(kind, X, k, seed) / np.where(d > 0, d, 1.0)  # a zero column stays zero
    Rn, piv = qrcp(P)
    r = rr_rank(Rn, tau)
    swaps = 0
    if f > 0:
        Rn, perm, swaps = strong_rrqr(Rn, r, f)
        piv = piv[perm]
        r = rr_rank(Rn, tau)
    Rout = np.asfortranarray(Rn[:r, :] * d[piv][None, :])
    Q = trsm_rows(np.asfortranarray(X[:, piv[:r]]), np.asfortranarray(Rout[:, :r])) if r else \
        np.zeros((m, 0), order="F")
    return dict(Q=Q, R=Rout, piv=piv, rank=r, Rn=Rn, swaps=swaps)


def rr_rcholqr2(X, k, seed, kind=GAUSSIAN, tau=1e-12, f=1.5):
    """RRRCholeskyQR2 (Section 4): Algorithm 7, then one Cholesky QR pass on
    the r kept columns as in Algorithm 3 steps 2-4: G = Q^T Q = R'^T R',
    Q <- Q R'^{-1}, R <- R' R.  Returns rr_rcholqr's dict with Q and R
    replaced and the Cholesky's status."""
    out = rr_rcholqr(X, k, seed, kind, tau, f)
    r = out["rank"]
    out["status"] = 0
    if r == 0:
        return out
    Rp, st = cholesky_upper(gram(out["Q"]))
    out["Q"] = trsm_rows(out["Q"], Rp)
    out["R"] = np.asfortranarray(np.triu(Rp) @ out["R"])
    out["status"] = int(st)
    return out


def qr_backward(Q, R, dQ, dR):
    """dX for X = Q R (positive-diagonal thin QR) given dQ, dR."""
    Q, R, dQ, dR = _f64(Q), _f64(R), _f64(dQ), _f64(dR)
    m, n = Q.shape
    dX = np.zeros((m, n), order="F")
    lib().orc_qr_backward(m, n, _ptr(Q), max(m, 1), _ptr(R), n, _ptr(dQ),
                          max(m, 1), _ptr(dR), n, _ptr(dX), max(m, 1))
    return dX
