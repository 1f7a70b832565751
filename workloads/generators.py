"""Seeded synthetic matrices (see the package docstring).  CPU / NumPy only."""

import math

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def haar(rng, m, n):
    """m x n matrix with orthonormal columns, Haar distributed (m >= n).

    QR of a Gaussian matrix with the signs of R's diagonal moved into Q
    (Mezzadri's correction), so the distribution is exactly Haar.
    """
    G = rng.standard_normal((m, n))
    Q, R = np.linalg.qr(G, mode="reduced")
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    return Q * sgn


def geometric_spectrum(n, q):
    """s_i = q^i for i = 1..n."""
    return q ** np.arange(1, n + 1, dtype=np.float64)


def power_spectrum(n, p):
    """s_i = i^-p for i = 1..n."""
    return np.arange(1, n + 1, dtype=np.float64) ** (-p)


def svd_matrix(m, n, s, seed, dtype=np.float64):
    """X = U diag(s) V^T with Haar U (m x r), V (n x r), r = len(s)."""
    rng = _rng(seed)
    r = len(s)
    U = haar(rng, m, r)
    V = haar(rng, n, r)
    X = (U * np.asarray(s)[None, :]) @ V.T
    return np.ascontiguousarray(X.astype(dtype))


def gaussian_exp_spectrum(r, flat=100, decay=0.8, floor=1e-5):
    """s_i = 1 for i <= flat, max(decay^(i - flat), floor) after (i = 1..r)."""
    i = np.arange(1, r + 1, dtype=np.float64)
    return np.where(i <= flat, 1.0, np.maximum(decay ** (i - flat), floor))


def gaussian_exp(m=1000, n=1000, seed=1006, dtype=np.float64, flat=100, decay=0.8,
                 floor=1e-5):
    """The Gaussian-exp matrix of the paper's experiments (section 6): Haar U,
    V and an exponentially decaying spectrum, flat for the first ``flat``
    values and floored at ``floor``; 1000 x 1000 in the paper."""
    r = min(m, n)
    return svd_matrix(m, n, gaussian_exp_spectrum(r, flat, decay, floor), seed, dtype)


def exact_rank(m, n, r, seed, dtype=np.float64, decay=0.9):
    """A matrix of exact rank r (Haar factors, s_i = decay^i)."""
    return svd_matrix(m, n, geometric_spectrum(r, decay), seed, dtype)


def _largest_remainder(total, weights):
    w = np.asarray(weights, dtype=np.float64)
    raw = total * w / w.sum()
    base = np.floor(raw).astype(np.int64)
    left = int(total - base.sum())
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:left]] += 1
    return base


def adversarial_gmm(m=100000, n=1000, sub_dim=200, n_comp=50, largest_frac=0.9,
                    dup_frac=0.05, dup_noise=1e-3, seed=1002, dtype=np.float32):
    """Adversarial Gaussian-mixture rows in a random subspace.

    * a Haar basis B (n x sub_dim) spans the data subspace;
    * component j (1..n_comp) has mean B (10 j e_j) -- distinct norms as in
      Example 4.1 -- and covariance B B^T (identity inside the subspace);
    * the component with the largest mean norm (j = n_comp) holds
      ``largest_frac`` of the base rows; component j < n_comp gets a share of
      the rest proportional to 1/j (largest-remainder rounding);
    * ``dup_frac`` of all rows are near-duplicates: a uniformly chosen base row
      x plus dup_noise ||x|| / sqrt(n) g with g ~ N(0, I_n);
    * rows are shuffled, then cast to ``dtype``.
    """
    rng = _rng(seed)
    assert 2 <= n_comp <= sub_dim <= n
    B = haar(rng, n, sub_dim)
    n_dup = int(round(dup_frac * m))
    n_base = m - n_dup
    n_big = int(round(largest_frac * n_base))
    small = _largest_remainder(n_base - n_big, 1.0 / np.arange(1, n_comp))
    sizes = np.concatenate([small, [n_big]])
    labels = np.repeat(np.arange(1, n_comp + 1), sizes)
    Z = rng.standard_normal((n_base, sub_dim))
    Z[np.arange(n_base), labels - 1] += 10.0 * labels
    base = Z @ B.T
    src = rng.integers(0, n_base, size=n_dup)
    xs = base[src]
    scale = dup_noise * np.linalg.norm(xs, axis=1, keepdims=True) / math.sqrt(n)
    dups = xs + scale * rng.standard_normal((n_dup, n))
    X = np.vstack([base, dups])
    X = X[rng.permutation(m)]
    return np.ascontiguousarray(X.astype(dtype))


def gmm_example41(n_clusters=100, cluster_size=20, n=500, seed=7, dtype=np.float64):
    """Example 4.1: means 10 j e_j (j = 1..k), covariance I, equal sizes."""
    rng = _rng(seed)
    assert n_clusters <= n
    m = n_clusters * cluster_size
    X = rng.standard_normal((m, n))
    j = np.repeat(np.arange(1, n_clusters + 1), cluster_size)
    X[np.arange(m), j - 1] += 10.0 * j
    return np.ascontiguousarray(X.astype(dtype))


def example23(m, k, r, alpha, n=None):
    """Example 2.3: X^T = [a_1 e_1 1^T, ..., a_k e_k 1^T] with m/k copies each.

    a_i = sqrt(alpha) for i <= r and 1 otherwise; n defaults to k.
    """
    assert m % k == 0 and r <= k
    n = k if n is None else n
    a = np.ones(k)
    a[:r] = math.sqrt(alpha)
    X = np.zeros((m, n))
    rep = m // k
    for i in range(k):
        X[i * rep:(i + 1) * rep, i] = a[i]
    return X


def kernel_blocks(count=4096, m_range=(64, 1024), n_range=(32, 256), h=0.5,
                  seed=1004, dtype=np.float32):
    """Gaussian-kernel blocks between separated 3-D clusters.

    Block i has m_i = round(exp U[ln m_lo, ln m_hi]) sources uniform in the
    unit cube and n_i = round(exp U[ln n_lo, ln n_hi]) targets uniform in the
    unit cube shifted by (2, 0, 0); X_i(p, q) = exp(-|x_p - y_q|^2 / h^2),
    evaluated in FP64 and cast to ``dtype``.  Returns a list of matrices.
    """
    rng = _rng(seed)
    lm = rng.uniform(math.log(m_range[0]), math.log(m_range[1]), size=count)
    ln = rng.uniform(math.log(n_range[0]), math.log(n_range[1]), size=count)
    ms = np.rint(np.exp(lm)).astype(np.int64)
    ns = np.rint(np.exp(ln)).astype(np.int64)
    out = []
    for i in range(count):
        xs = rng.uniform(0.0, 1.0, size=(ms[i], 3))
        ys = rng.uniform(0.0, 1.0, size=(ns[i], 3)) + np.array([2.0, 0.0, 0.0])
        d2 = ((xs[:, None, :] - ys[None, :, :]) ** 2).sum(-1)
        out.append(np.ascontiguousarray(np.exp(-d2 / (h * h)).astype(dtype)))
    return out


def random_features(m=1000000, n=4096, dim=64, n_comp=20, seed=1005,
                    dtype=np.float32, chunk=65536):
    """cos(x Omega + c): x from a GMM in R^dim (means N(0, I), covariance
    0.25 I, equal weights), Omega ~ N(0, 1/dim) (dim x n), c ~ U[0, 2 pi)^n.
    Generated in row chunks."""
    rng = _rng(seed)
    means = rng.standard_normal((n_comp, dim))
    Om = rng.standard_normal((dim, n)) / math.sqrt(dim)
    c = rng.uniform(0.0, 2.0 * math.pi, size=n)
    X = np.empty((m, n), dtype=dtype)
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        comp = rng.integers(0, n_comp, size=r1 - r0)
        x = means[comp] + 0.5 * rng.standard_normal((r1 - r0, dim))
        X[r0:r1] = np.cos(x @ Om + c).astype(dtype)
    return X


# The five workload configurations (m x n, tolerance, block size, dtype).
CONFIGS = {
    "svd_geometric_fp64": dict(m=2000, n=500, eps=1e-2, b=16, dtype="f64", seed=1001),
    "adversarial_gmm_fp32": dict(m=100000, n=1000, eps=1e-3, b=64, dtype="f32", seed=1002),
    "svd_power_bf16": dict(m=200000, n=2048, eps=1e-4, b=128, dtype="f32", seed=1003),
    "kernel_blocks_batched": dict(count=4096, eps=1e-6, dtype="f32", seed=1004),
    # eps-rank at 1e-3 is close to n for this generator: fixed rank k = 2048
    "random_features_large": dict(m=1000000, n=4096, eps=1e-3, b=256, dtype="f32", seed=1005,
                                  k_max=2048, fixed_rank=True),
}


def config_matrix(name, m=None, n=None):
    """The input matrix of a single-ID configuration, optionally resized."""
    cfg = CONFIGS[name]
    m = cfg["m"] if m is None else m
    n = cfg["n"] if n is None else n
    if name == "svd_geometric_fp64":
        return svd_matrix(m, n, geometric_spectrum(min(m, n), 0.9), cfg["seed"], np.float64)
    if name == "adversarial_gmm_fp32":
        sub = min(200, n)
        comp = min(50, sub)
        return adversarial_gmm(m, n, sub_dim=sub, n_comp=comp, seed=cfg["seed"])
    if name == "svd_power_bf16":
        return svd_matrix(m, n, power_spectrum(min(m, n), 1.5), cfg["seed"], np.float32)
    if name == "random_features_large":
        return random_features(m, n, seed=cfg["seed"])
    raise KeyError(name)
