"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random numbers and shapes them into raw series,
queries and filter weights.  It holds none of the search method's arithmetic:
no normalisation, no distances, no summaries.  Everything it returns is raw
fp32 (or int) data that the library and the oracle each process on their own.

Workloads follow the paper's experimental setup (Section "Evaluation Setup"):
random-walk collections built from N(0, 1) steps, query sets made of uniformly
drawn collection series with Gaussian noise added, and training queries with a
noise level drawn at random from a range.  The paper's real datasets are not
available; these synthetic sets stand in for them.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "random_walk",
    "random_walk_device",
    "random_walk_device_chunks",
    "noisy_queries_device",
    "gaussian_mixture",
    "noisy_queries",
    "mlp_weights",
    "WORKLOADS",
]


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_walk(n: int, m: int, seed: int, chunk: int = 262144) -> np.ndarray:
    """Raw random-walk series x_t = sum_{u<=t} e_u with e ~ N(0, 1), as fp32 [n, m].

    Generated in chunks (each chunk from its own child seed) so that large
    collections never hold more than one chunk of fp64 draws at a time.
    """
    out = np.empty((n, m), dtype=np.float32)
    children = np.random.SeedSequence(seed).spawn((n + chunk - 1) // chunk)
    for c, ss in enumerate(children):
        lo = c * chunk
        hi = min(n, lo + chunk)
        steps = _rng(ss).standard_normal((hi - lo, m))
        np.cumsum(steps, axis=1, out=steps)
        out[lo:hi] = steps
    return out


def _chunk_steps(n: int, m: int, seed: int, chunk: int, c: int, device):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed * 1_000_003 + c)
    lo = c * chunk
    hi = min(n, lo + chunk)
    return lo, hi, torch.randn((hi - lo, m), generator=g, device=device, dtype=torch.float32)


def random_walk_device(n: int, m: int, seed: int, device="cuda", chunk: int = 1 << 20):
    """Raw random walks generated on the GPU: x_t = sum_{u<=t} e_u with e ~ N(0, 1)
    from torch's Philox generator, fp32 [n, m] on `device`.  Chunk c (rows
    c*chunk ..) draws from its own seed, so any chunk can be regenerated alone
    (random_walk_device_chunks).  For collections too large to draw on the host
    in reasonable time; a different recipe from random_walk (NumPy PCG64)."""
    import torch
    out = torch.empty((n, m), dtype=torch.float32, device=device)
    for lo, hi, x in random_walk_device_chunks(n, m, seed, device, chunk):
        out[lo:hi] = x
    return out


def random_walk_device_chunks(n: int, m: int, seed: int, device="cuda", chunk: int = 1 << 20):
    """Yields (lo, hi, rows lo..hi of random_walk_device as a device tensor)."""
    import torch
    for c in range((n + chunk - 1) // chunk):
        lo, hi, steps = _chunk_steps(n, m, seed, chunk, c, device)
        yield lo, hi, torch.cumsum(steps, dim=1)


def noisy_queries_device(data, nq: int, sigma, seed: int):
    """noisy_queries for a device collection: nq distinct rows drawn uniformly
    (torch's generator, seeded) plus noise of standard deviation sigma *
    std(row) (population std; sigma a scalar or a (lo, hi) range drawn per
    query).  Returns (queries fp32 [nq, m] on the device, rows int64 [nq],
    levels fp64 [nq]) with rows and levels on the host."""
    import torch
    n, m = data.shape
    dev = data.device
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    rows = torch.randperm(n, generator=g, device=dev)[:nq]
    if isinstance(sigma, tuple):
        levels = sigma[0] + (sigma[1] - sigma[0]) * torch.rand((nq,), generator=g, device=dev, dtype=torch.float64)
    else:
        levels = torch.full((nq,), float(sigma), dtype=torch.float64, device=dev)
    base = data[rows].to(torch.float64)
    scale = base.std(dim=1, unbiased=False) * levels
    noise = torch.randn((nq, m), generator=g, device=dev, dtype=torch.float64)
    q = (base + scale[:, None] * noise).to(torch.float32)
    return q, rows.cpu().numpy(), levels.cpu().numpy()


def gaussian_mixture(n: int, m: int, n_comp: int, spread: float, seed_means: int,
                     seed_members: int, chunk: int = 262144) -> np.ndarray:
    """Series drawn from a Gaussian mixture: x = mu_c + N(0, spread^2), fp32 [n, m].

    Component means have N(0, 1) entries; each series picks its component
    uniformly.  Produces strongly clustered collections whose tree leaves are
    ragged in size.
    """
    means = _rng(seed_means).standard_normal((n_comp, m))
    out = np.empty((n, m), dtype=np.float32)
    children = np.random.SeedSequence(seed_members).spawn((n + chunk - 1) // chunk)
    for c, ss in enumerate(children):
        lo = c * chunk
        hi = min(n, lo + chunk)
        g = _rng(ss)
        comp = g.integers(0, n_comp, size=hi - lo)
        out[lo:hi] = means[comp] + spread * g.standard_normal((hi - lo, m))
    return out


def noisy_queries(data: np.ndarray, nq: int, sigma, seed_rows: int, seed_noise: int,
                  rows: np.ndarray | None = None):
    """Queries = collection series drawn uniformly without replacement + Gaussian noise.

    `sigma` is the noise level relative to each series' own scale: the noise
    added to row x has standard deviation sigma * std(x), which is the same as
    adding N(0, sigma^2) to the z-normalised series (z-normalisation is
    invariant to positive affine maps).  `sigma` may be a scalar, an array of
    per-query levels, or a (lo, hi) tuple, in which case each query draws its
    level uniformly from [lo, hi] (the paper's training-query recipe).

    Returns (queries fp32 [nq, m], source rows int64 [nq], levels fp64 [nq]).
    """
    n, m = data.shape
    if rows is None:
        rows = _rng(seed_rows).choice(n, size=nq, replace=False).astype(np.int64)
    g = _rng(seed_noise)
    if isinstance(sigma, tuple):
        levels = g.uniform(sigma[0], sigma[1], size=nq)
    else:
        levels = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (nq,)).copy()
    base = data[rows].astype(np.float64)
    scale = base.std(axis=1) * levels
    q = base + scale[:, None] * g.standard_normal((nq, m))
    return q.astype(np.float32), rows, levels


def mlp_weights(n_filters: int, m: int, h: int, seed: int, out_bias: float = 0.0) -> np.ndarray:
    """Seeded filter weights packed per filter as [W1 (h*m, i-major), b1 (h), w2 (h), b2].

    W1 is stored input-major: element (i, j) (input i, hidden unit j) sits at
    i*h + j.  Entries are uniform in +-1/sqrt(fan_in) (Kaiming-uniform with
    the default gain), so hidden activations stay O(1) for z-normalised input.
    Returns fp32 [n_filters, h*m + 2h + 1].
    """
    g = _rng(seed)
    w = np.empty((n_filters, h * m + 2 * h + 1), dtype=np.float32)
    a1 = 1.0 / np.sqrt(m)
    a2 = 1.0 / np.sqrt(h)
    w[:, : h * m] = g.uniform(-a1, a1, size=(n_filters, h * m))
    w[:, h * m: h * m + h] = g.uniform(-a1, a1, size=(n_filters, h))
    w[:, h * m + h: h * m + 2 * h] = g.uniform(-a2, a2, size=(n_filters, h))
    w[:, -1] = out_bias + g.uniform(-a2, a2, size=n_filters)
    return w


def cnn_weights(n_filters: int, C: int, seed: int, out_bias: float = 0.0) -> np.ndarray:
    """Seeded CNN filter weights packed per filter as
    [W1 (C, 3) | b1 (C) | W2 (C, C, 3) | b2 (C) | w3 (C) | b3], each layer
    uniform in +-1/sqrt(fan_in) (fan-in 3, 3C and C).  Returns fp32
    [n_filters, 3C^2 + 6C + 1]."""
    g = _rng(seed)
    P = 3 * C * C + 6 * C + 1
    w = np.empty((n_filters, P), dtype=np.float32)
    a1, a2, a3 = 1.0 / np.sqrt(3.0), 1.0 / np.sqrt(3.0 * C), 1.0 / np.sqrt(C)
    w[:, : 4 * C] = g.uniform(-a1, a1, size=(n_filters, 4 * C))
    w[:, 4 * C: 5 * C + 3 * C * C] = g.uniform(-a2, a2, size=(n_filters, C + 3 * C * C))
    w[:, 5 * C + 3 * C * C:] = g.uniform(-a3, a3, size=(n_filters, C + 1))
    w[:, -1] += out_bias
    return w


# Named workloads: the shapes and seeds every test and benchmark uses.
WORKLOADS = {
    # small plain-search case: exact 1-NN with lower-bound pruning only
    "rw20k": dict(kind="random_walk", n=20_000, m=256, seed=1001, capacity=1_000,
                  split="median", nq=100, q_rows_seed=1002, q_noise_seed=1003, sigma=0.1, k=1),
    # learned-filter case: 1M series, leaf capacity 10k, k=1, target recall 0.99
    "rw1m": dict(kind="random_walk", n=1_000_000, m=256, seed=2001, capacity=10_000,
                 split="median", n_calib=500, calib_seed=2004, test_seeds=(2005, 2006, 2007),
                 sigmas=(0.05, 0.1, 0.2), nq=1_000, k=1, target=0.99, train_seed=2002,
                 train_sigma=(0.05, 0.2)),
    # precision case: 10M series, bf16 scan with fp32 rerank of the top-4k, k=10
    "rw10m": dict(kind="random_walk", n=10_000_000, m=256, seed=3001, capacity=10_000,
                  split="median", nq=1_024, k=10, target=0.99, n_calib=500, calib_seed=3004,
                  test_seed=3005, train_seed=3002, sigmas=(0.05, 0.1, 0.2),
                  train_sigma=(0.05, 0.2)),
    # serving case: 50M random walks generated on the GPU (about 77 GB resident
    # as fp32 + bf16), leaf capacity 10k, mixed k and recall targets
    "rw50m": dict(kind="random_walk_device", n=50_000_000, m=256, seed=5001, capacity=10_000,
                  split="median", n_calib=500, calib_seed=5004, train_seed=5002, train_sigma=(0.05, 0.2),
                  sigma=0.1, test_seed=5005, ks=(1, 10, 100), targets=(0.90, 0.95, 0.99), mix_seed=5003,
                  nq=1_024, rates=(2_000, 5_000, 10_000, 20_000)),
    # the same collection and queries in an iSAX (MESSI) tree: 8 segments, 8-bit symbols
    "rw50m_isax": dict(kind="random_walk_device", n=50_000_000, m=256, seed=5001, capacity=10_000,
                       split="isax", segments=8, n_calib=500, calib_seed=5004, train_seed=5002,
                       train_sigma=(0.05, 0.2), sigma=0.1, test_seed=5005, ks=(1, 10, 100),
                       targets=(0.90, 0.95, 0.99), mix_seed=5003, nq=1_024, rates=(2_000, 5_000, 10_000, 20_000)),
    # ragged-leaf case: 25M length-96 Gaussian-mixture series, midpoint splits
    "gm25m": dict(kind="gaussian_mixture", n=25_000_000, m=96, n_comp=1_000, spread=0.3,
                  seed_means=4001, seed_members=4002, capacity=10_000, split="midpoint",
                  nq=4_096, q_seed=4003, sigma=0.1, ks=(1, 10, 50), target=0.99, n_calib=500,
                  calib_seed=4004, train_seed=4005, train_sigma=(0.05, 0.2)),
}
