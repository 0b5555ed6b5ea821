"""Seeded synthetic key sets (numpy PCG64).  Data only: nothing here computes
any part of the sorting method.

The paper sorts 200-500 MB of 64-bit floats drawn from uniform, normal and
log-normal distributions (Sec. 4.1, Datasets); the named workloads below keep
those shapes at fixed sizes, plus a skewed Gaussian mixture with duplicates,
heavy-tailed integer keys and a piecewise-uniform set with many breakpoints.
"""
from __future__ import annotations

import numpy as np

WORKLOADS = ("uniform", "lognormal", "gauss_mix", "zipf_u64", "piecewise_uniform")


def uniform(n: int, seed: int = 0) -> np.ndarray:
    """float64 keys i.i.d. Uniform[0, 1)."""
    return np.random.default_rng(seed).random(n)


def lognormal(n: int, seed: int = 1, sigma: float = 2.0) -> np.ndarray:
    """float64 keys i.i.d. LogNormal(0, sigma)."""
    return np.random.default_rng(seed).lognormal(0.0, sigma, n)


def gauss_mix(n: int, seed: int = 2) -> np.ndarray:
    """float64 keys from a skewed mixture of 8 Gaussians (weights
    Dirichlet(0.3), means U[-1e6, 1e6], standard deviations log-uniform in
    [1, 1e4]), then 1% of positions overwritten with copies of other keys."""
    rng = np.random.default_rng(seed)
    w = rng.dirichlet([0.3] * 8)
    mu = rng.uniform(-1e6, 1e6, 8)
    sd = 10.0 ** rng.uniform(0.0, 4.0, 8)
    c = rng.choice(8, n, p=w)
    x = mu[c] + sd[c] * rng.standard_normal(n)
    d = n // 100
    if d:
        dst = rng.choice(n, d, replace=False)
        src = rng.integers(0, n, d)
        x[dst] = x[src]
    return x


def zipf_u64(n: int, seed: int = 3, s: float = 1.1, limit: int = 1 << 40) -> np.ndarray:
    """uint64 keys k - 1 with k ~ Zipf(s), redrawn while k > limit, so keys lie
    in [0, limit)."""
    rng = np.random.default_rng(seed)
    k = rng.zipf(s, n)
    bad = k > limit
    while bad.any():
        k[bad] = rng.zipf(s, int(bad.sum()))
        bad = k > limit
    return (k - 1).astype(np.uint64)


def piecewise_uniform(n: int, seed: int = 4, breakpoints: int = 10_000,
                      chunk: int = 10_000_000) -> np.ndarray:
    """float64 keys from a piecewise-uniform density on [0, 1): sorted random
    breakpoints, segment masses 10**U[-4, 0] normalised; drawn in fixed chunks
    so the sequence does not depend on memory limits."""
    rng = np.random.default_rng(seed)
    bp = np.sort(rng.random(breakpoints))
    edges = np.concatenate([[0.0], bp, [1.0]])
    mass = 10.0 ** rng.uniform(-4.0, 0.0, breakpoints + 1)
    p = mass / mass.sum()
    out = np.empty(n, np.float64)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        seg = rng.choice(breakpoints + 1, b - a, p=p)
        lo = edges[seg]
        out[a:b] = lo + (edges[seg + 1] - lo) * rng.random(b - a)
    return out


def noisy_uniform(n: int, noise: float, seed: int = 5, mu: float = 0.5, sd: float = 0.1) -> np.ndarray:
    """Uniform [0, 1) keys with a fraction `noise` replaced by Normal(mu, sd)
    keys (the paper's changing-distribution experiment, Sec. 4, Exp-3: a model
    trained on uniform data sorts uniform + normal mixes)."""
    rng = np.random.default_rng(seed)
    x = rng.random(n)
    k = int(round(noise * n))
    if k:
        pos = rng.choice(n, k, replace=False)
        x[pos] = rng.normal(mu, sd, k)
    return x


def make(name: str, n: int, seed: int | None = None) -> np.ndarray:
    fn = {"uniform": uniform, "lognormal": lognormal, "gauss_mix": gauss_mix,
          "zipf_u64": zipf_u64, "piecewise_uniform": piecewise_uniform}[name]
    return fn(n) if seed is None else fn(n, seed)


# Named configurations: (workload, n, hidden width, form, fit sample fraction).
CONFIGS = {
    "uniform_1e6_fp32_h32": ("uniform", 10 ** 6, 32, "fp32", 0.01),
    "lognormal_1e8_fp32_h32": ("lognormal", 10 ** 8, 32, "fp32", 0.01),
    "gauss_mix_1e8_bf16_h64": ("gauss_mix", 10 ** 8, 64, "bf16", 0.01),
    "zipf_u64_1e7_fit_h64": ("zipf_u64", 10 ** 7, 64, "fp32", 0.10),
    "piecewise_uniform_1e9_bf16_h64": ("piecewise_uniform", 10 ** 9, 64, "bf16", 0.01),
}


def edge_keys(seed: int = 7) -> np.ndarray:
    """Small float64 set with signed zeros, subnormals, infinities, NaNs of
    both signs and payloads, duplicates and extreme magnitudes."""
    rng = np.random.default_rng(seed)
    special = np.array([0.0, -0.0, 5e-324, -5e-324, 2.2250738585072014e-308,
                        np.inf, -np.inf, 1.7976931348623157e308, -1.7976931348623157e308,
                        1.0, 1.0, 1.0, -1.0, 0.5, 0.5], np.float64)
    nans = np.array([0x7FF8000000000000, 0xFFF8000000000000, 0x7FF0000000000001,
                     0xFFF0000000000123], np.uint64).view(np.float64)
    body = rng.standard_normal(200)
    x = np.concatenate([special, nans, body, body[:20]])
    return x[rng.permutation(x.size)]
