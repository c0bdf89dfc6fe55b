"""Seeded generators for X = U diag(sigma) V^T (see the package docstring)."""
import numpy as np

# Stream tags: each random stream gets its own (seed, tag, chunk) key.
TAG_U, TAG_V, TAG_DQ, TAG_DR, TAG_SHAPES = 0x55, 0x56, 0x51, 0x52, 0x53
CHUNK = 1 << 16


def _rng(seed, tag, chunk=0):
    return np.random.Generator(np.random.Philox(
        np.random.SeedSequence([int(seed), int(tag), int(chunk)])))


def spectrum(n, sigma_min):
    """sigma_i = sigma_min^{i/(n-1)}, i = 0..n-1 (largest 1, smallest sigma_min)."""
    if n == 1:
        return np.ones(1)
    e = np.arange(n, dtype=np.float64) / (n - 1)
    return np.power(float(sigma_min), e)


def haar_square(n, seed):
    """Haar-distributed n x n orthogonal matrix (QR of a Gaussian, sign fix)."""
    G = _rng(seed, TAG_V).standard_normal((n, n))
    Qv, Rv = np.linalg.qr(G)
    d = np.sign(np.diag(Rv))
    d[d == 0] = 1.0
    return Qv * d


def _mixing(m, n, sigma_min, seed, gram):
    """M = (G^T G)^{-1/2} diag(sigma) V^T from the accumulated Gram of G."""
    lam, W = np.linalg.eigh(gram)
    T = (W / np.sqrt(lam)) @ W.T
    V = haar_square(n, seed)
    return T @ (spectrum(n, sigma_min)[:, None] * V.T)


def make_x(m, n, sigma_min, seed=0, dtype=np.float64):
    """X (m x n, Fortran order) with singular values spectrum(n, sigma_min).

    Deterministic for a given (m, n, sigma_min, seed) on any machine with
    the same numpy; G is drawn in chunks of 65536 rows (one stream each)."""
    nchunk = (m + CHUNK - 1) // CHUNK
    gram = np.zeros((n, n))
    for c in range(nchunk):
        rows = min(CHUNK, m - c * CHUNK)
        G = _rng(seed, TAG_U, c).standard_normal((rows, n))
        gram += G.T @ G
    M = _mixing(m, n, sigma_min, seed, gram)
    X = np.empty((m, n), dtype=dtype, order="F")
    for c in range(nchunk):
        rows = min(CHUNK, m - c * CHUNK)
        G = _rng(seed, TAG_U, c).standard_normal((rows, n))
        X[c * CHUNK:c * CHUNK + rows, :] = (G @ M).astype(dtype)
    return X


def make_x_torch(m, n, sigma_min, seed=0, dtype=None, device="cuda"):
    """Same construction drawn on a torch device (for multi-GB benchmark
    inputs).  Returns a column-major tensor: shape (m, n), stride (1, m).
    Uses torch's own seeded generator, so values differ from make_x."""
    import torch
    dtype = dtype or torch.float64
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1000003 + TAG_U)
    # Column-major m x n is the transpose of a row-major n x m buffer.
    Gt = torch.empty((n, m), dtype=torch.float64, device=device)
    step = 1 << 22
    for r0 in range(0, m, step):
        r1 = min(m, r0 + step)
        Gt[:, r0:r1].normal_(generator=g)
    gram = (Gt @ Gt.T).cpu().numpy()
    M = torch.from_numpy(_mixing(m, n, sigma_min, seed, gram)).to(device)
    Xt = torch.empty((n, m), dtype=dtype, device=device)
    for r0 in range(0, m, step):
        r1 = min(m, r0 + step)
        Xt[:, r0:r1] = (M.T @ Gt[:, r0:r1]).to(dtype)
    del Gt
    return Xt.T  # (m, n) view, column-major


def make_cotangents(m, n, seed=0):
    """dQ ~ N(0,1) (m x n) and dR = triu(N(0,1)) (n x n), Fortran order."""
    dQ = np.asfortranarray(_rng(seed, TAG_DQ).standard_normal((m, n)))
    dR = np.asfortranarray(np.triu(_rng(seed, TAG_DR).standard_normal((n, n))))
    return dQ, dR


def batched_shapes(count, seed=0, m_lo=2000, m_hi=200000,
                   n_choices=(16, 32, 64, 96, 128)):
    """Instance shapes for the batched workload: m uniform in [m_lo, m_hi],
    n uniform over n_choices, k = 3n."""
    r = _rng(seed, TAG_SHAPES)
    ms = r.integers(m_lo, m_hi + 1, size=count)
    ns = r.choice(np.asarray(n_choices), size=count)
    return [(int(a), int(b), int(3 * b)) for a, b in zip(ms, ns)]
