"""Pins for the FP64 CPU oracle: each routine is checked against something
other than itself -- an independent library implementation, LAPACK, mpmath,
exact distributions, closed forms, or the bounds of Theorem 5.2.

Section/equation references are to Balabanov, "Randomized Cholesky QR
factorizations".
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

import synth

U64 = 2.0 ** -53
G, RD, CS, ID = 0, 1, 2, 99


# ----------------------------------------------------------------- Philox
PIN_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Exposed : rocrand_device::philox4x32_10_engine {
  using rocrand_device::philox4x32_10_engine::ten_rounds;
};
int main() {
  Exposed e;
  unsigned c[4], k[2];
  while (scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    uint4 r = e.ten_rounds(uint4{c[0], c[1], c[2], c[3]}, uint2{k[0], k[1]});
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


def test_philox_matches_independent_library(orc, tmp_path):
    """Philox4x32-10 (Salmon et al. SC'11) against rocRAND's separately
    written header implementation, compiled as a host program."""
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(hdr) or shutil.which("g++") is None:
        pytest.skip("rocRAND header or g++ not available")
    src = tmp_path / "pin.cpp"
    src.write_text(PIN_SRC)
    exe = tmp_path / "pin"
    subprocess.run(["g++", "-O1", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                    str(src), "-o", str(exe)], check=True)
    rng = np.random.default_rng(7)
    cases = [[0] * 6, [0xffffffff] * 6]
    cases += rng.integers(0, 2 ** 32, size=(3000, 6), dtype=np.uint64).tolist()
    # structured counters as used by the sketch: (row lo, row hi, block, tag)
    for j in [0, 1, 2 ** 32 - 1, 2 ** 32, 10 ** 6 - 1]:
        for blk in [0, 1, 299]:
            cases.append([j & 0xffffffff, j >> 32, blk, 0x47415553, 1, 0])
    inp = "\n".join(" ".join("%x" % v for v in c) for c in cases) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        ref = [int(w, 16) for w in line.split()]
        assert orc.philox4x32_10(c[:4], c[4:]) == ref, c


def test_rademacher_bit_layout(orc):
    """Theta(i, j) is one bit of the Philox draw for (block j >> 7, row i):
    offset r = 32 q + 4 t + e within the block reads bit 8 e + t of word q,
    bit 1 meaning -1.  Checked entry by entry against Philox words from the
    library-pinned generator, on blocks far from the origin too."""
    seed = 0x0123456789ABCDEF
    for j0 in (0, 128 * 5 + 0, (1 << 40) + 256):
        th = orc.theta_block(RD, 300, j0 + 128, seed, 250, 4, j0, 128)
        for ii in range(4):
            b = j0 >> 7
            w = orc.philox4x32_10([b & 0xffffffff, b >> 32, 250 + ii, 0x52414445],
                                  [seed & 0xffffffff, seed >> 32])
            for r in range(128):
                q, t, e = r >> 5, (r & 31) >> 2, r & 3
                want = -1.0 if (w[q] >> (8 * e + t)) & 1 else 1.0
                assert th[ii, r] == want, (j0, ii, r)


def test_philox_bits_uniform(orc):
    """Rademacher entries are single Philox bits: chi-square over 2^16
    counters of the four-bit nibbles, and bit balance."""
    th = orc.theta_block(RD, 128, 4096, 12345, 0, 128, 0, 4096)
    bits = (th < 0).astype(np.int64)            # bit 1 -> -1
    assert abs(bits.mean() - 0.5) < 4 * 0.5 / math.sqrt(bits.size)
    nib = bits.reshape(-1, 4) @ np.array([1, 2, 4, 8])
    counts = np.bincount(nib, minlength=16)
    chi2 = scipy.stats.chisquare(counts).pvalue
    assert chi2 > 1e-4


# -------------------------------------------------------- Gaussian transform
def test_ln_matches_mpmath(orc):
    mp = pytest.importorskip("mpmath")
    mp.mp.prec = 120
    rng = np.random.default_rng(1)
    xs = list(rng.random(3000)) + [U64, 2 * U64, 1.0, 0.5, 0.70710678118654757,
                                  0.7071067811865475, 1.4142135623730951 / 2,
                                  np.nextafter(1.0, 0), 5e-324, 1e-310, 3.0, 1e300]
    xs += list(np.exp(-rng.random(2000) * 36.0))
    worst = 0.0
    for x in xs:
        x = float(x)
        if x <= 0:
            continue
        got = orc.ln(x)
        ref = mp.log(mp.mpf(x))
        ulp = math.ulp(float(ref)) if float(ref) != 0 else 5e-324
        err = abs(mp.mpf(got) - ref) / ulp
        worst = max(worst, float(err))
    assert worst <= 2.0, worst


def test_sincos2pi_matches_mpmath(orc):
    mp = pytest.importorskip("mpmath")
    mp.mp.prec = 120
    rng = np.random.default_rng(2)
    bs = [0, 1, 2 ** 50, 2 ** 51, 2 ** 52, 3 * 2 ** 51, 2 ** 53 - 1, 2 ** 51 - 1,
          2 ** 50 - 1, 2 ** 50 + 1]
    bs += [int(v) for v in rng.integers(0, 2 ** 53, size=3000, dtype=np.int64)]
    for b in bs:
        s, c = orc.sincos2pi_dyadic(b)
        ang = 2 * mp.pi * mp.mpf(b) / mp.mpf(2) ** 53
        assert abs(mp.mpf(s) - mp.sin(ang)) <= 4 * U64, b
        assert abs(mp.mpf(c) - mp.cos(ang)) <= 4 * U64, b


def test_gaussian_entries_are_standard_normal(orc):
    """Box-Muller output (Section 2: i.i.d. Gaussian entries) against the
    exact N(0,1) law: Kolmogorov-Smirnov and the first four moments."""
    z = orc.theta_block(G, 201, 6000, 99, 0, 201, 0, 6000).ravel()
    assert z.size == 201 * 6000
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-4
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / n)
    assert abs(scipy.stats.skew(z)) < 5 * math.sqrt(6 / n)
    assert abs(scipy.stats.kurtosis(z)) < 5 * math.sqrt(24 / n)
    # neighbouring rows (the cos/sin pair of one draw) are uncorrelated
    t = orc.theta_block(G, 2, 200000, 5, 0, 2, 0, 200000)
    assert abs(np.corrcoef(t[0], t[1])[0, 1]) < 5 / math.sqrt(200000)


def test_gaussian_odd_k_uses_cos_of_last_pair(orc):
    a = orc.theta_block(G, 7, 50, 3, 0, 7, 0, 50)
    b = orc.theta_block(G, 8, 50, 3, 0, 8, 0, 50)
    assert np.array_equal(a, b[:7])  # rows depend on (j, row), never on k


def test_countsketch_hash_and_isometry(orc):
    k = 37
    h = np.array([orc.countsketch_hash(k, 11, j)[0] for j in range(40000)])
    s = np.array([orc.countsketch_hash(k, 11, j)[1] for j in range(40000)])
    assert h.min() >= 0 and h.max() < k
    assert scipy.stats.chisquare(np.bincount(h, minlength=k)).pvalue > 1e-4
    assert abs(s.mean()) < 5 / math.sqrt(s.size)
    th = orc.theta_block(CS, k, 300, 4, 0, k, 0, 300)
    assert np.all(np.count_nonzero(th, axis=0) == 1)
    # E ||Theta x||^2 = ||x||^2 over seeds
    x = np.random.default_rng(0).standard_normal((300, 1))
    vals = [np.sum((orc.theta_block(CS, k, 300, sd, 0, k, 0, 300) @ x) ** 2)
            for sd in range(400)]
    assert abs(np.mean(vals) / np.sum(x ** 2) - 1) < 0.05


def test_dense_embeddings_are_isometric_in_mean(orc):
    """E ||Theta x||^2 = ||x||^2 for the rescaled Gaussian and Rademacher
    embeddings of Section 2."""
    x = np.random.default_rng(3).standard_normal((500, 1))
    for kind in (G, RD):
        vals = []
        for sd in range(60):
            th = orc.theta_block(kind, 64, 500, sd, 0, 64, 0, 500)
            vals.append(np.sum((orc.sketch_scale(kind, 64) * th @ x) ** 2))
        assert abs(np.mean(vals) / np.sum(x ** 2) - 1) < 0.06


# ---------------------------------------------------------- sketch P = Theta X
@pytest.mark.parametrize("kind,k", [(G, 31), (G, 32), (RD, 130), (CS, 17)])
def test_sketch_equals_materialised_product(orc, kind, k):
    m, n = 700, 9
    X = np.asfortranarray(np.random.default_rng(4).standard_normal((m, n)))
    P = orc.sketch(kind, X, k, 77)
    th = orc.theta_block(kind, k, m, 77, 0, k, 0, m)
    ref = orc.sketch_scale(kind, k) * (th @ X)
    bound = 2 * m * U64 * orc.sketch_scale(kind, k) * (np.abs(th) @ np.abs(X))
    assert np.all(np.abs(P - ref) <= bound + 1e-300)


def test_sketch_exact_dot_mpmath(orc):
    mp = pytest.importorskip("mpmath")
    mp.mp.prec = 200
    m, n, k = 300, 3, 6
    X = np.asfortranarray(np.random.default_rng(5).standard_normal((m, n)))
    P = orc.sketch(G, X, k, 8)
    th = orc.theta_block(G, k, m, 8, 0, k, 0, m)
    sc = mp.mpf(1) / mp.sqrt(k)
    for i in range(k):
        for c in range(n):
            exact = sc * mp.fsum(mp.mpf(th[i, j]) * mp.mpf(X[j, c]) for j in range(m))
            scale = float(np.abs(th[i]) @ np.abs(X[:, c])) / math.sqrt(k)
            assert abs(mp.mpf(P[i, c]) - exact) <= 2 * m * U64 * scale


def test_identity_sketch_is_copy(orc):
    X = np.asfortranarray(np.random.default_rng(6).standard_normal((40, 5)))
    assert np.array_equal(orc.sketch(ID, X, 40, 0), X)


# ------------------------------------------------------------ small FP64 QR
def _lapack_qr_posdiag(A):
    Qn, Rn = np.linalg.qr(A)
    d = np.sign(np.diag(Rn))
    d[d == 0] = 1
    return Qn * d, d[:, None] * Rn


@pytest.mark.parametrize("k,n", [(1, 1), (5, 5), (30, 10), (150, 50), (97, 33)])
def test_householder_matches_lapack(orc, k, n):
    P = np.asfortranarray(np.random.default_rng(k * 100 + n).standard_normal((k, n)))
    R, S, st = orc.householder_qr(P)
    assert st == 0
    Sr, Rr = _lapack_qr_posdiag(P)
    assert np.all(np.diag(R) > 0)
    assert np.array_equal(np.tril(R, -1), np.zeros_like(R))
    cond = np.linalg.cond(P)
    assert np.linalg.norm(R - Rr) <= 50 * n * U64 * cond * np.linalg.norm(Rr)
    assert np.linalg.norm(S - Sr) <= 50 * n * U64 * cond * math.sqrt(n)
    # Assumption (eq. ass2): orthonormal S and small P - S R
    assert np.linalg.norm(S.T @ S - np.eye(n)) <= 10 * k * n * U64
    assert np.linalg.norm(P - S @ R) <= 10 * k * n * U64 * np.linalg.norm(P)


def test_householder_extreme_column_scales(orc):
    """Columns of magnitude 1e-200 and 1e+200 (sums of squares that underflow
    or overflow in FP64): R matches LAPACK's (whose reflectors guard their
    norms) column by column, and equals the R of the rescaled matrix exactly
    (a power-of-two column scaling commutes with Householder QR)."""
    rng = np.random.default_rng(31)
    P = np.asfortranarray(rng.standard_normal((60, 12)))
    e = np.array([0, -664, 0, 664, -10, 0, 300, -700, 0, 0, 2, -1])   # 2^-664 ~ 1e-200
    Ps = np.asfortranarray(P * np.ldexp(1.0, e)[None, :])
    R, S, st = orc.householder_qr(Ps)
    assert st == 0
    R0, S0, st0 = orc.householder_qr(P)
    assert st0 == 0
    assert np.array_equal(R, R0 * np.ldexp(1.0, e)[None, :])
    assert np.array_equal(S, S0)
    _, Rr = _lapack_qr_posdiag(Ps)
    for c in range(12):
        assert np.linalg.norm(R[:, c] - Rr[:, c]) <= 1e-13 * np.linalg.norm(Rr[:, c])


def test_householder_zero_column_flags_rank(orc):
    P = np.asfortranarray(np.random.default_rng(9).standard_normal((20, 4)))
    P[:, 2] = 0.0
    _, _, st = orc.householder_qr(P)
    assert st == 1


# ---------------------------------------------------- forward substitution
def test_row_substitution_matches_lapack_and_is_backward_stable(orc):
    rng = np.random.default_rng(10)
    m, n = 500, 40
    X = np.asfortranarray(rng.standard_normal((m, n)))
    _, R = _lapack_qr_posdiag(rng.standard_normal((n + 20, n)) @ np.diag(
        np.logspace(0, -6, n)))
    R = np.asfortranarray(R)
    Q = orc.trsm_rows(X, R)
    ref = scipy.linalg.solve_triangular(R, X.T, trans="T", lower=False).T
    cond = np.linalg.cond(R)
    assert np.linalg.norm(Q - ref) <= 10 * n * U64 * cond * np.linalg.norm(ref)
    # Higham Thm 8.5 as used in Section 5.1: |x_i - q_i R| <= 1.1 u n |q_i||R|
    lhs = np.abs(X - Q @ R)
    rhs = 1.1 * U64 * n * (np.abs(Q) @ np.abs(R))
    assert np.all(lhs <= rhs + 1e-300)


# --------------------------------------------------------- Cholesky, R product
def test_cholesky_matches_lapack(orc):
    rng = np.random.default_rng(11)
    A = rng.standard_normal((200, 30))
    Gm = np.asfortranarray(A.T @ A)
    Rp, st = orc.cholesky_upper(Gm)
    assert st == 0
    Lr = np.linalg.cholesky(Gm)
    assert np.linalg.norm(Rp - Lr.T) <= 1e-13 * np.linalg.norm(Lr)
    assert np.array_equal(np.tril(Rp, -1), np.zeros_like(Rp))


def test_cholesky_breakdown_reports_column(orc):
    Gm = np.eye(5)
    Gm[3, 3] = -1.0
    _, st = orc.cholesky_upper(np.asfortranarray(Gm))
    assert st == 1003


def test_triu_product_matches_matmul(orc):
    rng = np.random.default_rng(12)
    A = np.triu(rng.standard_normal((17, 17)))
    B = np.triu(rng.standard_normal((17, 17)))
    C = orc.triu_product(A, B)
    assert np.allclose(C, A @ B, rtol=0, atol=1e-13)
    assert np.array_equal(np.tril(C, -1), np.zeros_like(C))


def test_gram_matches_matmul(orc):
    Q = np.asfortranarray(np.random.default_rng(13).standard_normal((3000, 12)))
    Gm = orc.gram(Q)
    assert np.allclose(Gm, Q.T @ Q, rtol=0, atol=3000 * U64 * 12 * 4)
    assert np.array_equal(Gm, Gm.T)


# ------------------------------------------------ whole algorithm: special cases
@pytest.mark.parametrize("kind", [G, RD, CS])
def test_two_pass_equals_lapack_thin_qr(orc, kind):
    """Algorithm 3 in exact arithmetic returns the unique positive-diagonal
    thin QR, whatever Theta is: compare with LAPACK at kappa = 1e3."""
    m, n = 3000, 20
    X = synth.make_x(m, n, 1e-3, seed=1)
    out = orc.rcholqr(X, 3 * n, 5, kind, passes=2)
    assert out["status"] == 0
    Qr, Rr = _lapack_qr_posdiag(X)
    assert np.linalg.norm(out["R"] - Rr) <= 1e-12 * np.linalg.norm(Rr)
    assert np.linalg.norm(out["Q"] - Qr) <= 1e-12 * np.linalg.norm(Qr)


def test_identity_sketch_reduces_to_householder(orc):
    """Theta = I (k = m): Algorithm 2 is Householder QR of X then Q = X R^-1."""
    m, n = 400, 12
    X = synth.make_x(m, n, 1e-4, seed=2)
    out = orc.rcholqr(X, m, 0, ID, passes=1)
    assert out["status"] == 0
    Qr, Rr = _lapack_qr_posdiag(X)
    assert np.linalg.norm(out["R"] - Rr) <= 1e-13 * np.linalg.norm(Rr)
    assert np.linalg.norm(out["Q"] - Qr) <= 1e-10
    assert np.linalg.norm(out["Q"].T @ out["Q"] - np.eye(n), 2) <= 1e-10


def test_single_column_closed_forms(orc):
    rng = np.random.default_rng(14)
    x = np.asfortranarray(rng.standard_normal((1000, 1)) * 3.0)
    two = orc.rcholqr(x, 3, 6, G, passes=2)
    assert abs(two["R"][0, 0] - np.linalg.norm(x)) <= 1e-13 * np.linalg.norm(x)
    assert np.allclose(two["Q"], x / np.linalg.norm(x), rtol=0, atol=1e-15)
    one = orc.rcholqr(x, 3, 6, G, passes=1)
    th = orc.theta_block(G, 3, 1000, 6, 0, 3, 0, 1000) / math.sqrt(3)
    r = np.linalg.norm(th @ x)
    assert abs(one["R"][0, 0] - r) <= 1e-13 * r
    assert np.allclose(one["Q"], x / r, rtol=1e-14, atol=0)


def test_orthonormal_input_gives_identity_r(orc):
    X = synth.make_x(2000, 16, 1.0, seed=3)     # sigma all ones: Q = X, R = I
    out = orc.rcholqr(X, 48, 1, G, passes=2)
    assert np.linalg.norm(out["R"] - np.eye(16)) <= 1e-13
    assert np.linalg.norm(out["Q"] - X) <= 1e-13


def test_diagonal_input(orc):
    d = np.array([3.0, -2.0, 0.5, 7.0])
    X = np.zeros((50, 4), order="F")
    X[:4, :4] = np.diag(d)
    out = orc.rcholqr(X, 12, 2, RD, passes=2)
    E = np.zeros((50, 4))
    E[:4, :4] = np.diag(np.sign(d))
    assert np.allclose(out["Q"], E, atol=1e-14)
    assert np.allclose(out["R"], np.diag(np.abs(d)), atol=1e-13)


def test_singular_values_of_r_are_sigma(orc):
    """X = U diag(sigma) V^T: R has the same singular values (Weyl)."""
    X = synth.make_x(5000, 30, 1e-6, seed=4)
    out = orc.rcholqr(X, 90, 3, G, passes=2)
    sv = np.linalg.svd(out["R"], compute_uv=False)
    assert np.all(np.abs(sv - synth.spectrum(30, 1e-6)) <= 1e-13)


# ------------------------------------------------- Theorem 5.2 invariants
def test_theorem_5_2_bounds_config_a(orc):
    """m=10000, n=50, k=150, sigma down to 1e-8, Gaussian, one pass."""
    m, n, k = 10000, 50, 150
    X = synth.make_x(m, n, 1e-8, seed=0)
    out = orc.rcholqr(X, k, 1, G, passes=1, want_s=True)
    assert out["status"] == 0
    Q, R, S = out["Q"], out["R"], out["S"]
    # eq. main1: ||X_j - (QR)_j|| <= 2.1 u n ||X_j||
    col = np.linalg.norm(X - Q @ R, axis=0) / np.linalg.norm(X, axis=0)
    assert col.max() <= 2.1 * U64 * n
    # eq. main3: ||S - Theta Q||_F <= 6.1 u n^1.5 kappa
    th = orc.theta_block(G, k, m, 1, 0, k, 0, m) / math.sqrt(k)
    kappa = np.linalg.cond(X / np.linalg.norm(X, axis=0))
    assert np.linalg.norm(S - th @ Q) <= 6.1 * U64 * n ** 1.5 * kappa
    # sketched orthonormality of Q (eq. sketchedcond, up to eq. main3)
    SQ = th @ Q
    assert np.linalg.norm(SQ.T @ SQ - np.eye(n), 2) <= 2 * 6.1 * U64 * n ** 1.5 * kappa
    # Corollary 2.2: cond(Q) = cond(Theta U) for an orthonormal basis U;
    # for k = 3n it concentrates near (1+sqrt(1/3))/(1-sqrt(1/3)) ~ 3.7
    assert np.linalg.cond(Q) <= 20


@pytest.mark.parametrize("kind", [G, RD, CS])
def test_two_pass_orthogonality_at_kappa_1e12(orc, kind):
    m, n = 20000, 40
    X = synth.make_x(m, n, 1e-12, seed=5)
    out = orc.rcholqr(X, 3 * n, 9, kind, passes=2)
    assert out["status"] == 0
    Q, R = out["Q"], out["R"]
    assert np.linalg.norm(Q.T @ Q - np.eye(n), 2) <= 1e-12
    col = np.linalg.norm(X - Q @ R, axis=0) / np.linalg.norm(X, axis=0)
    assert col.max() <= 1e-13


def test_status_codes(orc):
    X = synth.make_x(500, 6, 1e-2, seed=6)
    Xz = X.copy()
    Xz[:, 3] = 0.0
    assert orc.rcholqr(Xz, 18, 1, G, passes=2)["status"] == 1
    Xn = X.copy()
    Xn[7, 2] = np.nan
    assert orc.rcholqr(Xn, 18, 1, G, passes=2)["status"] == 2


# ---------------------------------------------------------------- adjoint
def _loss(orc, X, dQ, dR, seed):
    o = orc.rcholqr(X, 3 * X.shape[1], seed, G, passes=2)
    return float(np.sum(o["Q"] * dQ) + np.sum(o["R"] * dR)), o


def test_adjoint_matches_finite_differences(orc):
    m, n = 2000, 16
    X = synth.make_x(m, n, 1e-2, seed=7)
    dQ, dR = synth.make_cotangents(m, n, seed=7)
    _, o = _loss(orc, X, dQ, dR, 1)
    dX = orc.qr_backward(o["Q"], o["R"], dQ, dR)
    E = np.asfortranarray(np.random.default_rng(8).standard_normal((m, n)))
    h = 1e-5 * np.linalg.norm(X) / np.linalg.norm(E)
    lp, _ = _loss(orc, X + h * E, dQ, dR, 1)
    lm, _ = _loss(orc, X - h * E, dQ, dR, 1)
    fd = (lp - lm) / (2 * h)
    an = float(np.sum(dX * E))
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_adjoint_matches_autograd_of_lapack_qr(orc):
    torch = pytest.importorskip("torch")
    m, n = 300, 10
    X = synth.make_x(m, n, 1e-3, seed=8)
    dQ, dR = synth.make_cotangents(m, n, seed=9)
    Xt = torch.tensor(np.ascontiguousarray(X), dtype=torch.float64, requires_grad=True)
    Qt, Rt = torch.linalg.qr(Xt)
    d = torch.sign(torch.diagonal(Rt)).detach()
    Qt, Rt = Qt * d, d[:, None] * Rt
    loss = (Qt * torch.tensor(dQ)).sum() + (Rt * torch.tensor(dR)).sum()
    loss.backward()
    o = orc.rcholqr(X, 3 * n, 2, G, passes=2)
    dX = orc.qr_backward(o["Q"], o["R"], dQ, dR)
    ref = Xt.grad.numpy()
    assert np.linalg.norm(dX - ref) <= 1e-10 * np.linalg.norm(ref)


def test_adjoint_single_column_closed_form(orc):
    rng = np.random.default_rng(15)
    x = rng.standard_normal((200, 1))
    r = np.linalg.norm(x)
    q = x / r
    qb = rng.standard_normal((200, 1))
    rb = np.array([[1.7]])
    dX = orc.qr_backward(q, np.array([[r]]), qb, rb)
    ref = (qb - q * (q.T @ qb)) / r + q * rb[0, 0]
    assert np.allclose(dX, ref, rtol=0, atol=1e-14)


# ----------------------------------------------------------------------------- Algorithm 5
@pytest.mark.parametrize("kind,k", [(G, 31), (G, 64), (RD, 130)])
def test_extractor_rows_follow_theta_rows(orc, kind, k):
    """Theta' = [Theta; L]: the rows of the (k + l)-row operator below k are
    the k-row operator's own rows (entries depend on the row index only)."""
    m, l = 300, 17
    a = orc.theta_block(kind, k, m, 4, 0, k, 0, m)
    b = orc.theta_block(kind, k + l, m, 4, 0, k + l, 0, m)
    assert np.array_equal(a, b[:k])
    L = orc.extractor(kind, k, l, m, 4)
    assert np.array_equal(L, b[k:] * orc.sketch_scale(kind, l))
    with pytest.raises(ValueError):
        orc.extractor(CS, k, l, m, 4)


@pytest.mark.parametrize("kind", [G, RD])
def test_reduced_equals_extractor_times_q(orc, kind):
    """Extracting before the solve (step 3 of Algorithm 5) gives L Q for the Q
    of Algorithm 2 with the same Theta; R is the same R bit for bit."""
    m, n, k, l = 3000, 12, 36, 9
    X = synth.make_x(m, n, 1e-3, seed=21)
    red = orc.reduced_rcholqr(X, k, l, 5, kind)
    one = orc.rcholqr(X, k, 5, kind, passes=1)
    assert red["status"] == 0 and one["status"] == 0
    assert np.array_equal(red["R"], one["R"])
    LQ = orc.extractor(kind, k, l, m, 5) @ one["Q"]
    assert np.linalg.norm(red["Z"] - LQ) <= 1e-11 * np.linalg.norm(LQ)


def test_reduced_is_invariant_under_power_of_two_column_scaling(orc):
    """X D with D = diag(2^e): P, Y scale by D exactly, R by D, so Z = Y R^{-1}
    is the same bits (catches a transposed or misplaced triangular factor)."""
    m, n, k, l = 800, 7, 21, 5
    X = synth.make_x(m, n, 1e-2, seed=22)
    D = 2.0 ** np.array([3, -5, 0, 7, -2, 1, -9], dtype=np.float64)
    a = orc.reduced_rcholqr(X, k, l, 8, RD)
    b = orc.reduced_rcholqr(X * D, k, l, 8, RD)
    assert np.array_equal(b["R"], a["R"] * D)
    assert np.array_equal(b["Z"], a["Z"])


def test_reduced_single_column_closed_form(orc):
    """n = 1: R = ||Theta x||, Z = L x / ||Theta x|| (scaled operators)."""
    m, k, l = 500, 9, 4
    x = np.asfortranarray(np.random.default_rng(3).standard_normal((m, 1)))
    red = orc.reduced_rcholqr(x, k, l, 2, G)
    th = orc.theta_block(G, k, m, 2, 0, k, 0, m) * orc.sketch_scale(G, k)
    r = np.linalg.norm(th @ x)
    assert abs(red["R"][0, 0] - r) <= 1e-14 * r
    z = (orc.extractor(G, k, l, m, 2) @ x) / r
    assert np.allclose(red["Z"], z, rtol=1e-13, atol=0)


# ----------------------------------------------------------------------------- Algorithm 7
def test_qrcp_matches_lapack_geqp3(orc):
    """Column-pivoted Householder against LAPACK's xGEQP3 (distinct norms:
    the same pivots; R equal up to row signs)."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((60, 20)) * np.logspace(0, 4, 20)[rng.permutation(20)]
    R, piv = orc.qrcp(A)
    _, Rl, pl = scipy.linalg.qr(A, mode="economic", pivoting=True)
    assert np.array_equal(piv, pl)
    assert np.allclose(R, np.abs(np.diag(Rl))[:, None] / np.diag(Rl)[:, None] * Rl,
                       rtol=1e-12, atol=1e-12 * np.abs(Rl).max())
    assert np.all(np.diag(R) >= 0)
    assert np.all(np.diff(np.diag(R)) <= 1e-12 * R[0, 0])  # non-increasing pivots


@pytest.mark.parametrize("kind", [G, RD])
def test_rr_rcholqr_finds_exact_rank(orc, kind):
    """X = U V of exact rank 7 (n = 16): r = 7, X Pi = Q R on all columns
    (the dropped ones within tau), Q well-conditioned."""
    rng = np.random.default_rng(9)
    m, n, rho, k = 4000, 16, 7, 48
    X = rng.standard_normal((m, rho)) @ rng.standard_normal((rho, n))
    X = np.asfortranarray(X * np.logspace(0, 3, n))
    out = orc.rr_rcholqr(X, k, 3, kind, tau=1e-10)
    assert out["rank"] == rho
    Q, R, piv = out["Q"], out["R"], out["piv"]
    assert np.linalg.cond(Q) <= 10
    XP = X[:, piv]
    err = np.linalg.norm(XP - Q @ R, axis=0) / np.linalg.norm(XP, axis=0)
    assert err.max() <= 1e-9


def test_colnorms_closed_forms(orc):
    """D of Algorithm 7: the 2-norm of each column, also where a plain sum of
    squares overflows or underflows -- a column of two equal entries v has
    norm sqrt(2)|v| for v = 1e200 and 1e-200, a zero column 0, and the norm
    is homogeneous, ||c x|| = |c| ||x||, for c = 1e170, 1e-170, -3."""
    X = np.array([[1e200, 1e-200, 0.0, 3.0], [1e200, -1e-200, 0.0, 4.0]])
    d = orc.colnorms(X)
    assert d[0] == pytest.approx(math.sqrt(2) * 1e200, rel=1e-15)
    assert d[1] == pytest.approx(math.sqrt(2) * 1e-200, rel=1e-15)
    assert d[2] == 0.0 and d[3] == pytest.approx(5.0, rel=1e-15)
    rng = np.random.default_rng(3)
    X0 = rng.standard_normal((1000, 6))
    for c in (1e170, 1e-170, -3.0):
        assert np.allclose(orc.colnorms(X0 * c), abs(c) * np.linalg.norm(X0, axis=0),
                           rtol=2e-15, atol=0.0)
    assert orc.colnorms(np.zeros((0, 3))).tolist() == [0.0, 0.0, 0.0]


def test_rr_rcholqr_is_column_scale_invariant(orc):
    """Algorithm 7 normalises X by D, so scaling columns by 1e170 and 1e-170
    leaves the rank, the pivots and Q as they were (to rounding)."""
    rng = np.random.default_rng(9)
    m, n, rho, k = 4000, 16, 7, 48
    X = np.asfortranarray(rng.standard_normal((m, rho)) @ rng.standard_normal((rho, n)))
    sc = np.ones(n)
    sc[0::3], sc[1::3] = 1e170, 1e-170
    a = orc.rr_rcholqr(X, k, 3, RD, tau=1e-10)
    b = orc.rr_rcholqr(np.asfortranarray(X * sc[None, :]), k, 3, RD, tau=1e-10)
    assert a["rank"] == b["rank"] == rho
    assert np.array_equal(a["piv"][:rho], b["piv"][:rho])
    assert np.linalg.norm(a["Q"] - b["Q"]) <= 1e-12 * np.linalg.norm(a["Q"])


def test_rr_rcholqr_full_rank_is_stable_beyond_cholesky(orc):
    """kappa = 1e14 (beyond what the Cholesky-based passes take): with a tiny
    tau every column is kept or the trailing part is below tau; Q stays
    well-conditioned and X Pi = Q R to ~u n."""
    m, n, k = 3000, 20, 60
    X = synth.make_x(m, n, 1e-14, seed=4)
    out = orc.rr_rcholqr(X, k, 2, G, tau=1e-15)
    Q, R, piv, r = out["Q"], out["R"], out["piv"], out["rank"]
    assert np.linalg.cond(Q) <= 20
    XP = X[:, piv]
    err = np.linalg.norm(XP[:, :r] - Q @ R[:, :r], axis=0) / np.linalg.norm(XP[:, :r], axis=0)
    assert err.max() <= 1e-12


def test_rr_rank_rule(orc):
    """Step 3: the least r with ||R[r:, r:]||_F <= tau ||R||_2."""
    R = np.diag([4.0, 2.0, 1e-3, 1e-9, 0.0])
    assert orc.rr_rank(R, 1e-2) == 2
    assert orc.rr_rank(R, 1e-8) == 3
    assert orc.rr_rank(R, 1e-12) == 4
    assert orc.rr_rank(R, 0.0) == 4
    assert orc.rr_rank(np.zeros((3, 3)), 1e-3) == 0


def test_rr_rcholqr2_full_rank_equals_householder_r(orc):
    """RRRCholeskyQR2 on a full-rank X (kappa 1e4): Q is orthonormal to
    working accuracy and, the positive-diagonal QR of X Pi being unique, R is
    LAPACK's Householder R of X[:, piv] with its rows made positive."""
    m, n, k = 3000, 24, 72
    X = synth.make_x(m, n, 1e-4, seed=6)
    out = orc.rr_rcholqr2(X, k, 4, G, tau=1e-14)
    assert out["rank"] == n and out["status"] == 0
    Q, R, piv = out["Q"], out["R"], out["piv"]
    assert np.linalg.norm(Q.T @ Q - np.eye(n), 2) <= 1e-14
    Rl = np.linalg.qr(X[:, piv], mode="r")
    Rl = np.sign(np.diag(Rl))[:, None] * Rl
    assert np.linalg.norm(R - Rl) <= 1e-12 * np.linalg.norm(Rl)
    # the pivots and rank are those of the single pass
    one = orc.rr_rcholqr(X, k, 4, G, tau=1e-14)
    assert np.array_equal(one["piv"], piv) and one["rank"] == n


def test_rr_rcholqr2_low_rank_restores_orthogonality(orc):
    """Exact rank 9 of n = 20: the single pass leaves cond(Q) of a few units;
    the second pass makes Q orthonormal to ~u and keeps X Pi = Q R."""
    rng = np.random.default_rng(12)
    m, n, rho, k = 5000, 20, 9, 60
    X = np.asfortranarray((rng.standard_normal((m, rho)) @ rng.standard_normal((rho, n)))
                          * np.logspace(0, 2, n))
    one = orc.rr_rcholqr(X, k, 8, RD, tau=1e-10)
    two = orc.rr_rcholqr2(X, k, 8, RD, tau=1e-10)
    assert one["rank"] == two["rank"] == rho
    assert np.linalg.norm(one["Q"].T @ one["Q"] - np.eye(rho), 2) > 1e-3
    Q, R = two["Q"], two["R"]
    assert np.linalg.norm(Q.T @ Q - np.eye(rho), 2) <= 1e-14
    XP = X[:, two["piv"]]
    err = np.linalg.norm(XP - Q @ R, axis=0) / np.linalg.norm(XP, axis=0)
    assert err.max() <= 1e-9


def _kahan(n, c):
    s = math.sqrt(1.0 - c * c)
    K = np.diag(s ** np.arange(n)) @ (np.eye(n) - c * np.triu(np.ones((n, n)), 1))
    return K * (1.0 - 1e-10) ** np.arange(n)[None, :]  # column pivoting keeps the order


def _ge_bound(n, k, f):
    return math.sqrt(1.0 + f * f * k * (n - k))


def test_strong_rrqr_reveals_the_kahan_rank(orc):
    """Kahan's matrix (n = 32, c = 0.285) defeats column pivoting: it keeps the
    natural order and leaves R[n-1, n-1] ~ 0.27 while sigma_n ~ 2e-4.  The
    strong RRQR swaps meet Gu and Eisenstat's bounds for k = n - 1:
    sigma_i(R11) >= sigma_i / b and sigma_j(R22) <= sigma_{k+j} b with
    b = sqrt(1 + f^2 k (n - k)), and R is the QR factor of K[:, perm]."""
    n, f = 32, 1.5
    K = _kahan(n, 0.285)
    sv = np.linalg.svd(K, compute_uv=False)
    R0, piv0 = orc.qrcp(K)
    assert np.array_equal(piv0, np.arange(n))
    assert R0[-1, -1] > 1e3 * sv[-1]
    R, perm, swaps = orc.strong_rrqr(R0, n - 1, f)
    assert swaps >= 1
    b = _ge_bound(n, n - 1, f)
    s11 = np.linalg.svd(R[:-1, :-1], compute_uv=False)
    assert np.all(s11 >= sv[:-1] / b)
    assert abs(R[-1, -1]) <= sv[-1] * b
    Rl = np.linalg.qr(K[:, perm], mode="r")
    Rl = np.sign(np.diag(Rl))[:, None] * Rl
    assert np.allclose(R, Rl, rtol=0, atol=1e-13)


@pytest.mark.parametrize("seed", [1, 3])
def test_strong_rrqr_bounds_on_a_graded_spectrum(orc, seed):
    """X = U diag(10^(-14 t)) V^T (n = 64, no gap): at k = the rule's rank the
    singular values of R11 and R22 after the swaps are within Gu and
    Eisenstat's factor of X's, and rr_rcholqr's Q and R factor X Pi."""
    rng = np.random.default_rng(seed)
    m, n, k = 4000, 64, 192
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    X = np.asfortranarray((U * np.logspace(0, -14, n)) @ V.T)
    out = orc.rr_rcholqr(X, k, seed, G, tau=1e-7)
    r, Rn = out["rank"], out["Rn"]
    assert out["swaps"] >= 1
    # Rn factors the normalised sketch; compare with its own singular values
    Pn = orc.sketch(G, X, k, seed) / np.linalg.norm(X, axis=0)
    sv = np.linalg.svd(Pn[:, out["piv"]], compute_uv=False)
    b = _ge_bound(n, r, 1.5)
    assert np.all(np.linalg.svd(Rn[:r, :r], compute_uv=False) >= sv[:r] / b * (1 - 1e-9))
    assert np.all(np.linalg.svd(Rn[r:, r:], compute_uv=False) <= sv[r:] * b * (1 + 1e-9) + 1e-15)
    Q, R, piv = out["Q"], out["R"], out["piv"]
    assert np.linalg.cond(Q) <= 10
    XP = X[:, piv]
    err = np.linalg.norm(XP - Q @ R) / np.linalg.norm(XP)
    assert err <= 1e-6


# ----------------------------------------------------------------------------- SRHT
@pytest.mark.parametrize("m", [1000, 300, 1])
def test_srht_theta_is_signed_sylvester_hadamard(orc, m):
    """Theta's raw entries are d_j H[s_i, j] with H scipy's Sylvester-Hadamard
    matrix of order m' = 2^ceil(log2 m), d_j = +-1 and s_i in [0, m')."""
    k, seed = 40, 7
    mp = 1 << orc.srht_log2(m)
    assert mp >= m and (mp == 1 or mp < 2 * m)
    th = orc.theta_block(orc.SRHT, k, m, seed, 0, k, 0, m)
    d = orc.srht_signs(seed, m)
    s = orc.srht_rows(seed, k, m)
    assert np.all(np.abs(d) == 1) and np.all((0 <= s) & (s < mp))
    assert np.array_equal(th, scipy.linalg.hadamard(mp)[s][:, :m] * d[None, :])
    # a block away from the origin equals the same rows of the full block
    if m == 1000:
        assert np.array_equal(orc.theta_block(orc.SRHT, k, m, seed, 5, 20, 130, 300),
                              th[5:25, 130:430])


@pytest.mark.parametrize("m,n", [(1000, 12), (513, 5), (1, 3)])
def test_srht_fast_transform_equals_the_dense_theta(orc, m, n):
    """The oracle's SRHT sketch (signs, fast Walsh-Hadamard transform of the
    zero-padded rows, sampling, 1/sqrt(k)) equals Theta X / sqrt(k) formed
    from the closed-form entries."""
    k = 3 * n
    X = np.random.default_rng(m).standard_normal((m, n))
    P = orc.sketch(orc.SRHT, X, k, 11)
    th = orc.theta_block(orc.SRHT, k, m, 11, 0, k, 0, m)
    assert np.allclose(P, th @ X / np.sqrt(k), rtol=0, atol=1e-13 * np.abs(X).sum(axis=0).max())


def test_srht_is_an_embedding_and_rcholqr_is_stable(orc):
    """Orthonormal U (m = 8192, n = 32): the singular values of Theta U lie in
    [1 - eps, 1 + eps] with eps ~ 0.6 at k = 3n, as for the Gaussian
    embedding; RCholeskyQR2 with the SRHT at kappa = 1e10 gives an orthonormal
    Q to ~u and R as LAPACK's Householder R."""
    U = synth.make_x(8192, 32, 1.0, seed=3)
    sv = np.linalg.svd(orc.sketch(orc.SRHT, U, 96, 5), compute_uv=False)
    assert sv.min() >= 0.3 and sv.max() <= 1.7
    X = synth.make_x(8192, 32, 1e-10, seed=4)
    out = orc.rcholqr(X, 96, 5, orc.SRHT, passes=2)
    assert out["status"] == 0
    Q, R = out["Q"], out["R"]
    assert np.linalg.norm(Q.T @ Q - np.eye(32), 2) <= 1e-13
    Rl = np.linalg.qr(X, mode="r")
    Rl = np.sign(np.diag(Rl))[:, None] * Rl
    for j in range(32):
        assert np.linalg.norm(R[:, j] - Rl[:, j]) <= 1e-6 * np.linalg.norm(X[:, j])


# ----------------------------------------------------------------------------- Algorithm 4
@pytest.mark.parametrize("widths,kind", [((16, 16, 16, 16), G), ((20, 7, 33), RD),
                                         ((1,) * 24, G), ((40,), CS)])
def test_col_rcholqr_equals_algorithm_2(orc, widths, kind):
    """Section 3.2: block by block, Algorithm 4 computes what Algorithm 2
    computes on the whole X (the C oracle's one-pass RCholeskyQR), up to
    rounding: same Q, S and R for a well-conditioned X; p = n is the
    column-by-column case."""
    n = sum(widths)
    m, k = 3000, 3 * n
    X = synth.make_x(m, n, 1e-3, seed=13)
    cuts = np.cumsum((0,) + widths)
    out = orc.col_rcholqr([X[:, a:b] for a, b in zip(cuts[:-1], cuts[1:])], k, 4, kind)
    ref = orc.rcholqr(X, k, 4, kind, passes=1, want_s=True)
    assert np.linalg.norm(out["R"] - ref["R"]) <= 1e-12 * np.linalg.norm(ref["R"])
    assert np.linalg.norm(out["Q"] - ref["Q"]) <= 1e-11 * np.linalg.norm(ref["Q"])
    assert np.linalg.norm(out["S"] - ref["S"]) <= 1e-12 * np.linalg.norm(ref["S"])
    # one projection per block: S keeps orthogonality to ~u kappa (kappa = 1e3)
    assert np.linalg.norm(out["S"].T @ out["S"] - np.eye(n), 2) <= 1e-11
    assert np.allclose(np.triu(out["R"]), out["R"], rtol=0, atol=0)
