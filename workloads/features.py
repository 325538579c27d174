"""Feature generators for the five workloads (see the package docstring)."""
import numpy as np


def normalize(x):
    """Row-wise L2 normalisation carried out in float32."""
    x = np.asarray(x, dtype=np.float32)
    nrm = np.sqrt(np.sum(x * x, axis=-1, keepdims=True, dtype=np.float32)).astype(np.float32)
    return (x / nrm).astype(np.float32)


def tiny_gallery(seed=1, d=16, n=128, noise=0.05, known=7):
    """Small ring workload: 128 templates around 128 random centres, one i.i.d.
    query and one query near centre `known` (the known answer)."""
    rng = np.random.default_rng(seed)
    q = normalize(rng.standard_normal(d))
    centres = normalize(rng.standard_normal((n, d)))
    X = normalize(centres + noise * rng.standard_normal((n, d)))
    q_known = normalize(centres[known] + noise * rng.standard_normal(d))
    return dict(query=q, query_known=q_known, known=known, gallery=X)


def face_gallery(seed=2, d=128, n=6144, noise=0.05, known=4321):
    """Face-scale workload: n i.i.d. Gaussian templates, a query near template
    `known` and an i.i.d. query."""
    rng = np.random.default_rng(seed)
    X = normalize(rng.standard_normal((n, d)))
    q_known = normalize(X[known] + noise * rng.standard_normal(d))
    q = normalize(rng.standard_normal(d))
    return dict(query=q, query_known=q_known, known=known, gallery=X)


def fingerprint_gallery(seed=3, d=16, n=1 << 20, identities=1000, noise=0.1, rows=None):
    """Large fingerprint-scale gallery from a clustered Gaussian mixture:
    template t belongs to identity t mod `identities`.  `rows` limits the
    generated rows (a prefix of the same stream) for sampled checks."""
    rng = np.random.default_rng(seed)
    centres = normalize(rng.standard_normal((identities, d)))
    q_id = int(rng.integers(identities))
    q = normalize(centres[q_id] + noise * rng.standard_normal(d))
    m = n if rows is None else min(n, rows)
    X = np.empty((m, d), dtype=np.float32)
    step = 1 << 16
    for lo in range(0, m, step):
        hi = min(m, lo + step)
        ids = np.arange(lo, hi) % identities
        X[lo:hi] = normalize(centres[ids] + noise * rng.standard_normal((hi - lo, d)))
    return dict(query=q, query_identity=q_id, gallery=X, identities=identities)


def mixed_batch(seed=4, dims=(16, 64, 128, 512), queries_per_dim=16,
                sizes=((200_000, 1_000), (100_000, 3_000), (50_000, 6_144), (20_000, 10_000)),
                scale_sizes=1.0):
    """Batched workload: per dimension two galleries of uneven size and
    `queries_per_dim` queries, each query matched against both galleries of
    its dimension.  `scale_sizes` shrinks every gallery for quick checks."""
    rng = np.random.default_rng(seed)
    galleries, queries = [], []
    for d, pair in zip(dims, sizes):
        for n in pair:
            n = max(1, int(n * scale_sizes))
            galleries.append(dict(d=d, X=normalize(rng.standard_normal((n, d)))))
        for _ in range(queries_per_dim):
            queries.append(dict(d=d, q=normalize(rng.standard_normal(d))))
    return dict(galleries=galleries, queries=queries)


def serving_galleries(seed=5, scale_sizes=1.0):
    """Sixteen resident galleries: twelve 128-dim and four 16-dim."""
    rng = np.random.default_rng(seed)
    s128 = [6144, 10_000, 20_000, 30_000, 50_000, 75_000, 100_000, 150_000,
            200_000, 300_000, 400_000, 500_000]
    s16 = [6144, 50_000, 200_000, 500_000]
    out = []
    for d, sizes in ((128, s128), (16, s16)):
        for n in sizes:
            n = max(1, int(n * scale_sizes))
            out.append(dict(d=d, X=normalize(rng.standard_normal((n, d)))))
    return out


def poisson_arrivals(seed, rate_qps, count, mix_128_to_16=3):
    """Arrival times (s) of a Poisson process and each request's dimension."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_qps, size=count)
    t = np.cumsum(gaps)
    dims = np.where(rng.random(count) < mix_128_to_16 / (mix_128_to_16 + 1.0), 128, 16)
    return t, dims, rng.integers(0, 1 << 30, size=count)
