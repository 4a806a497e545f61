"""Seeded synthetic inputs for graph construction.

This module only draws random numbers: it holds none of the graph-construction
arithmetic, so both the plain CPU reference under ``oracle/`` and the GPU
library's tests and benchmarks can use it without sharing method code.

The evaluation datasets of the paper (SIFT1M, GIST1M, DEEP1M; Section 4.1) are
not available here. The generators below produce data with the same shapes and
similar statistics, and stand in for them:

* ``mixture``   -- isotropic Gaussian mixture, centres U[-1,1]^d (10k x 128 case).
* ``sift_like`` -- integer-valued features in [0, 255] from a cluster mixture with
                   per-dimension skew (half-normal magnitudes, rounded); every
                   squared L2 distance at d <= 128 is then exact in FP32.
* ``gist_like`` -- Gaussian mixture whose per-coordinate variance decays as 1/k.
* ``angular``   -- unit vectors from a von Mises-Fisher-like mixture (for IP).
* ``binary``    -- 0/1 rows (Hamming distances: exact ties everywhere; tests only).

Every generator is deterministic in its seeds and independent of chunking:
rows are drawn in fixed blocks of ``_BLOCK`` rows, each from its own stream.
"""
from __future__ import annotations

import numpy as np

_BLOCK = 65536


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def _labels(rng: np.random.Generator, m: int, k: int) -> np.ndarray:
    return rng.integers(0, k, size=m)


def _blocks(n: int):
    for b0 in range(0, n, _BLOCK):
        yield b0 // _BLOCK, b0, min(n, b0 + _BLOCK)


# ---------------------------------------------------------------- mixture (10k x 128)
def mixture(n: int, d: int = 128, k: int = 50, sigma: float = 0.15,
            seed: int = 1, stream: int = 0) -> np.ndarray:
    """Isotropic Gaussian mixture: centres ~ U[-1,1]^d (drawn from ``seed``),
    labels uniform, x = c + sigma * N(0, I). ``stream`` selects an independent
    sample from the same mixture (0 = base points, 1 = held-out queries...)."""
    centres = _rng(seed, 0xC0).uniform(-1.0, 1.0, size=(k, d))
    out = np.empty((n, d), dtype=np.float32)
    for bi, b0, b1 in _blocks(n):
        r = _rng(seed, 0xD0 + stream, bi)
        lab = _labels(r, b1 - b0, k)
        out[b0:b1] = (centres[lab] + sigma * r.standard_normal((b1 - b0, d))).astype(np.float32)
    return out


# ---------------------------------------------------------------- SIFT-like (integer valued)
def sift_like(n: int, d: int = 128, k: int = 1000, seed: int = 11,
              stream: int = 0) -> np.ndarray:
    """Integer-valued float32 features in [0, 255].

    Per-dimension spread s_j ~ U[8, 64]; cluster centre mu_cj = |N(0,1)| * s_j
    (half-normal); x_j = clip(round(|mu_cj + 0.35 s_j N(0,1)|), 0, 255)."""
    rc = _rng(seed, 0xC1)
    s = rc.uniform(8.0, 64.0, size=d)
    mu = np.abs(rc.standard_normal((k, d))) * s
    out = np.empty((n, d), dtype=np.float32)
    for bi, b0, b1 in _blocks(n):
        r = _rng(seed, 0xD1 + stream, bi)
        lab = _labels(r, b1 - b0, k)
        x = np.abs(mu[lab] + 0.35 * s * r.standard_normal((b1 - b0, d)))
        out[b0:b1] = np.clip(np.rint(x), 0, 255).astype(np.float32)
    return out


# ---------------------------------------------------------------- GIST-like (decaying spectrum)
def gist_like(n: int, d: int = 960, k: int = 1000, seed: int = 21,
              stream: int = 0) -> np.ndarray:
    """Mixture with per-coordinate variance lambda_k = 1/k (k = 1..d):
    mu_c = sqrt(lambda) * N(0, I); x = mu_c + 0.5 sqrt(lambda) * N(0, I)."""
    lam_sqrt = 1.0 / np.sqrt(np.arange(1, d + 1, dtype=np.float64))
    mu = _rng(seed, 0xC2).standard_normal((k, d)) * lam_sqrt
    out = np.empty((n, d), dtype=np.float32)
    for bi, b0, b1 in _blocks(n):
        r = _rng(seed, 0xD2 + stream, bi)
        lab = _labels(r, b1 - b0, k)
        out[b0:b1] = (mu[lab] + 0.5 * lam_sqrt * r.standard_normal((b1 - b0, d))).astype(np.float32)
    return out


# ---------------------------------------------------------------- angular (unit vectors)
def angular(n: int, d: int = 100, k: int = 2000, seed: int = 31,
            stream: int = 0) -> np.ndarray:
    """Unit vectors: mean directions m_c = N(0,I)/|.|; x = normalize(m_c + 0.75 N(0,I)/sqrt(d))."""
    m = _rng(seed, 0xC3).standard_normal((k, d))
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    out = np.empty((n, d), dtype=np.float32)
    for bi, b0, b1 in _blocks(n):
        r = _rng(seed, 0xD3 + stream, bi)
        lab = _labels(r, b1 - b0, k)
        x = m[lab] + 0.75 * r.standard_normal((b1 - b0, d)) / np.sqrt(d)
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out[b0:b1] = x.astype(np.float32)
    return out


# ---------------------------------------------------------------- binary (heavy ties)
def binary(n: int, d: int = 16, seed: int = 41, stream: int = 0) -> np.ndarray:
    """0/1-valued float32 rows, coordinate j set with probability p_j ~ U[0.2, 0.8].
    Squared L2 distances are Hamming distances (integers 0..d), so most of them
    tie exactly and, at small d, some rows repeat: a stress case for the
    (key, id) order of every list the construction keeps."""
    pj = _rng(seed, 0xC5).uniform(0.2, 0.8, size=d)
    out = np.empty((n, d), dtype=np.float32)
    for bi, b0, b1 in _blocks(n):
        r = _rng(seed, 0xD5 + stream, bi)
        out[b0:b1] = (r.random((b1 - b0, d)) < pj).astype(np.float32)
    return out


# ---------------------------------------------------------------- named workloads
#: name -> (generator, kwargs, metric, R). Sizes are the full ones; callers may
#: ask for fewer rows of the same distribution.
WORKLOADS = {
    "mixture10k_d128": dict(gen=mixture, kw=dict(d=128, k=50, sigma=0.15, seed=1),
                            n=10_000, nq=1_000, metric=0, R=32),
    "siftlike1m_d128": dict(gen=sift_like, kw=dict(d=128, k=1000, seed=11),
                            n=1_000_000, nq=10_000, metric=0, R=32),
    "gistlike1m_d960": dict(gen=gist_like, kw=dict(d=960, k=1000, seed=21),
                            n=1_000_000, nq=10_000, metric=0, R=48),
    "angular1.2m_d100": dict(gen=angular, kw=dict(d=100, k=2000, seed=31),
                             n=1_200_000, nq=10_000, metric=1, R=32),
}


def workload(name: str, n: int | None = None, nq: int | None = None):
    """Return (points, queries, metric, R) for a named workload; ``n``/``nq``
    override the row counts (same distribution, same seeds)."""
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    nq = w["nq"] if nq is None else nq
    X = w["gen"](n, stream=0, **w["kw"])
    Q = w["gen"](nq, stream=1, **w["kw"])
    return X, Q, w["metric"], w["R"]


def random_pool(n: int, R: int, K: int, seed: int) -> np.ndarray:
    """Distinct random neighbour ids (no self) for every vertex: an (n, R) int32
    array whose first K columns are ids and the rest -1. Ordering of the ids
    is left to the caller (keys are not computed here)."""
    r = _rng(seed, 0xE0)
    ids = np.full((n, R), -1, dtype=np.int32)
    for v in range(n):
        c = r.choice(n - 1, size=K, replace=False)
        c = c + (c >= v)
        ids[v, :K] = c
    return ids


# ------------------------------------------------------------ serving stream
def serving_requests(count: int = 512, seed: int = 5, n_max: int = 200_000):
    """Descriptors of the serving workload: request i has n log-uniform in
    [2,000, n_max] (200,000 by default), d from {96, 128, 384, 768}, 20-500
    clusters, L2 or IP (50/50), R from {16, 32}, and its own data seed
    1000 + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(2_000), np.log(n_max))))
        out.append(dict(n=n, d=int(rng.choice([96, 128, 384, 768])),
                        k=int(rng.integers(20, 501)), metric=int(rng.integers(0, 2)),
                        R=int(rng.choice([16, 32])), seed=1000 + i))
    return out


def serving_data_gpu(n: int, d: int, k: int, metric: int, seed: int, nq: int = 100,
                     sigma: float = 0.15, device="cuda"):
    """One serving request's points and queries, generated on the device with
    a seeded torch generator: a Gaussian mixture (centres U[-1,1]^d, spread
    sigma); inner-product rows are unit-normalised. Returns (X, Q) float32."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    cen = torch.rand((k, d), generator=gen, device=device) * 2.0 - 1.0

    def draw(m):
        lab = torch.randint(0, k, (m,), generator=gen, device=device)
        x = cen[lab] + sigma * torch.randn((m, d), generator=gen, device=device)
        if metric == 1:
            x = x / x.norm(dim=1, keepdim=True)
        return x.contiguous()

    return draw(n), draw(nq)
