"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds only random-number recipes; none of the similarity
method's arithmetic lives here.  The GPU library and the CPU oracle are both
fed from it, and neither imports the other.

The paper measures on MNIST (60k x 784 grey-level images), NORB, CIFAR-10 and
TIMIT (Sec. 4.4), none of which is available here; the recipes below stand in
for them with the same shapes and value ranges.  All draws use
numpy.random.Generator(PCG64(seed)).

  mixture_isotropic   N=2000, D=50: 10 isotropic unit-variance Gaussians with
                      centres ~ N(0, 16 I), exactly N/10 points each, shuffled.
  image_like          N=70000, D=784: 10 non-negative prototypes with 60% zero
                      pixels (non-zero pixels ~ U(0,1)), x = clip(proto +
                      N(0, 0.1^2), 0, 1), N/10 points per prototype, shuffled.
  mixture_anisotropic N=1e6, D=128: 50 Gaussian clusters, centres ~ N(0, 16 I),
                      covariance Q diag(lambda) Q^T with lambda ~ U[0.1, 4] and
                      Q the sign-fixed QR factor of a Gaussian matrix.
  activity_stream     stand-in for the sensor stream of Sec. 8 (52 readings
                      every 100 ms, 24 labelled activities): a time-ordered
                      sequence of activity segments (length ~ U[200, 900]
                      readings, activity drawn uniformly from 24 centres ~
                      N(0, 9 I)); within a segment each reading is the centre
                      plus an AR(1) drift (coefficient 0.98, innovation
                      N(0, 0.2^2 I)) plus N(0, 0.5^2 I) sensor noise.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 20251203


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _balanced_labels(rng: np.random.Generator, n: int, n_clusters: int) -> np.ndarray:
    lab = np.arange(n) % n_clusters
    rng.shuffle(lab)
    return lab


def mixture_isotropic(n: int = 2000, d: int = 50, n_clusters: int = 10, centre_std: float = 4.0,
                      seed: int = BASE_SEED + 1) -> np.ndarray:
    rng = _rng(seed)
    centres = rng.normal(0.0, centre_std, size=(n_clusters, d))
    lab = _balanced_labels(rng, n, n_clusters)
    x = centres[lab] + rng.normal(0.0, 1.0, size=(n, d))
    return x.astype(np.float32)


def image_prototypes(d: int = 784, n_clusters: int = 10, zero_frac: float = 0.6,
                     seed: int = BASE_SEED + 2) -> np.ndarray:
    rng = _rng(seed)
    proto = rng.uniform(0.0, 1.0, size=(n_clusters, d))
    proto[rng.uniform(0.0, 1.0, size=(n_clusters, d)) < zero_frac] = 0.0
    return proto


def image_like(n: int = 70000, d: int = 784, n_clusters: int = 10, noise: float = 0.1,
               seed: int = BASE_SEED + 2, noise_seed: int | None = None) -> np.ndarray:
    """Image-shaped points; ``noise_seed`` draws fresh points from the same prototypes."""
    proto = image_prototypes(d, n_clusters, seed=seed)
    rng = _rng(seed * 7 + 1 if noise_seed is None else noise_seed)
    lab = _balanced_labels(rng, n, n_clusters)
    out = np.empty((n, d), np.float32)
    step = 8192
    for s in range(0, n, step):
        e = min(n, s + step)
        blk = proto[lab[s:e]] + rng.normal(0.0, noise, size=(e - s, d))
        np.clip(blk, 0.0, 1.0, out=blk)
        out[s:e] = blk
    return out


def mixture_anisotropic(n: int = 1_000_000, d: int = 128, n_clusters: int = 50, centre_std: float = 4.0,
                        lam_lo: float = 0.1, lam_hi: float = 4.0, seed: int = BASE_SEED + 4) -> np.ndarray:
    rng = _rng(seed)
    centres = rng.normal(0.0, centre_std, size=(n_clusters, d))
    lab = _balanced_labels(rng, n, n_clusters)
    out = np.empty((n, d), np.float32)
    for m in range(n_clusters):
        g = rng.normal(size=(d, d))
        q, r = np.linalg.qr(g)
        q = q * np.sign(np.diag(r))[None, :]
        lam = rng.uniform(lam_lo, lam_hi, size=d)
        rows = np.nonzero(lab == m)[0]
        z = rng.normal(size=(rows.size, d))
        out[rows] = (centres[m] + (z * np.sqrt(lam)[None, :]) @ q.T).astype(np.float32)
    return out


def activity_stream(n: int = 12000, d: int = 52, n_activities: int = 24, seed: int = BASE_SEED + 5) -> np.ndarray:
    """Time-ordered readings (row t is the reading at tick t)."""
    rng = _rng(seed)
    centres = rng.normal(0.0, 3.0, size=(n_activities, d))
    out = np.empty((n, d), np.float32)
    t = 0
    drift = np.zeros(d)
    while t < n:
        length = int(rng.integers(200, 901))
        act = int(rng.integers(0, n_activities))
        for s in range(t, min(n, t + length)):
            drift = 0.98 * drift + rng.normal(0.0, 0.2, size=d)
            out[s] = centres[act] + drift + rng.normal(0.0, 0.5, size=d)
        t += length
    return out


def small_cases(seed: int = BASE_SEED + 9):
    """Assorted small seeded inputs (ragged sizes, odd D) for parity tests."""
    rng = _rng(seed)
    cases = []
    for n, d in [(97, 3), (130, 17), (257, 64), (300, 127), (515, 50), (1000, 128), (777, 785)]:
        cases.append(rng.normal(size=(n, d)).astype(np.float32))
    return cases


CONFIGS = {
    1: dict(name="mixture10_N2000_D50", n=2000, d=50, perplexity=30.0, k=90),
    2: dict(name="imagelike_N70000_D784", n=70000, d=784, perplexity=30.0, k=90),
    3: dict(name="imagelike_N70000_D784_bf16", n=70000, d=784, perplexity=30.0, k=90),
    4: dict(name="aniso50_N1000000_D128_fp8", n=1_000_000, d=128, perplexity=50.0, k=150),
}


def config_data(cfg: int) -> np.ndarray:
    if cfg == 1:
        return mixture_isotropic()
    if cfg in (2, 3):
        return image_like()
    if cfg == 4:
        return mixture_anisotropic()
    raise ValueError(cfg)
