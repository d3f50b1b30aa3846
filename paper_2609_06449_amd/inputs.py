"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This module holds random-number recipes only: it does no transform
arithmetic, and neither the oracle nor the GPU library is imported here.
The paper has no datasets; these stand in for its workloads with the shapes
and value distributions of the configured problems:

* uniform:     real and imaginary parts i.i.d. U[-1, 1]
* normal:      real and imaginary parts i.i.d. N(0, 1)
* loguniform:  |x| = 10**U[-4, 4], arg x ~ U[0, 2*pi)  (dynamic-range stress)

All draws use ``numpy.random.default_rng(seed)`` (PCG64) in float64, the
real parts drawn first, then the imaginary parts (or magnitudes, then
phases), and are rounded once to complex64.  Large inputs are drawn in
chunks of the same stream so that host memory stays near one complex64
buffer.
"""
from __future__ import annotations

import numpy as np

_CHUNK = 1 << 22


def _fill(rng, n: int, draw) -> np.ndarray:
    out = np.empty(n, dtype=np.float32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        out[s:e] = draw(rng, e - s)
    return out


def uniform(N: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = np.empty(N, dtype=np.complex64)
    x.real = _fill(rng, N, lambda r, n: r.uniform(-1.0, 1.0, n))
    x.imag = _fill(rng, N, lambda r, n: r.uniform(-1.0, 1.0, n))
    return x


def normal(N: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = np.empty(N, dtype=np.complex64)
    x.real = _fill(rng, N, lambda r, n: r.standard_normal(n))
    x.imag = _fill(rng, N, lambda r, n: r.standard_normal(n))
    return x


def loguniform(N: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    mag = np.empty(N, dtype=np.float64)
    for s in range(0, N, _CHUNK):
        e = min(N, s + _CHUNK)
        mag[s:e] = 10.0 ** rng.uniform(-4.0, 4.0, e - s)
    x = np.empty(N, dtype=np.complex64)
    for s in range(0, N, _CHUNK):
        e = min(N, s + _CHUNK)
        ph = rng.uniform(0.0, 2.0 * np.pi, e - s)
        x[s:e] = (mag[s:e] * np.exp(1j * ph)).astype(np.complex64)
    return x


def batch_sizes(count: int = 4096, seed: int = 6, kmin: int = 8, kmax: int = 20) -> np.ndarray:
    """Transform lengths N_i = 2**k_i with k_i ~ U{kmin..kmax} (inclusive)."""
    rng = np.random.default_rng(seed)
    ks = rng.integers(kmin, kmax + 1, size=count)
    return (np.int64(1) << ks.astype(np.int64)).astype(np.int64)


def batch_inputs(sizes, seed: int = 6) -> np.ndarray:
    """Packed batch: transform i (normal entries, its own child seed) at offset
    sum_{j<i} N_j of one complex64 array."""
    sizes = np.asarray(sizes, dtype=np.int64)
    children = np.random.SeedSequence(seed).spawn(len(sizes))
    out = np.empty(int(sizes.sum()), dtype=np.complex64)
    off = 0
    for n, ss in zip(sizes.tolist(), children):
        rng = np.random.default_rng(ss)
        out[off:off + n].real = rng.standard_normal(n)
        out[off:off + n].imag = rng.standard_normal(n)
        off += n
    return out


# The configured problems: (name, N1, N2, p, b, generator, seed).
CONFIGS = {
    "n4096_64x64_b4":  dict(N1=64, N2=64, p=4, b=4, gen="uniform", seed=1),
    "n2p24_4096x4096_b16":  dict(N1=4096, N2=4096, p=64, b=16, gen="normal", seed=2),
    "n2p28_16384x16384_b4": dict(N1=1 << 14, N2=1 << 14, p=256, b=4, gen="normal", seed=3),
    "n2p28_8192x32768_b2": dict(N1=1 << 13, N2=1 << 15, p=128, b=2, gen="normal", seed=4),
    # the 2^28 shapes with their literal bases (mixed-radix: 2^14 = 16^3 * 4,
    # 2^13 = 8^4 * 2)
    "n2p28_16384x16384_b16": dict(N1=1 << 14, N2=1 << 14, p=256, b=16, gen="normal", seed=3),
    "n2p28_8192x32768_b8": dict(N1=1 << 13, N2=1 << 15, p=128, b=8, gen="normal", seed=4),
    "n2p24_4096x4096_b16_loguniform": dict(N1=4096, N2=4096, p=64, b=16, gen="loguniform", seed=5),
    "n2p26_4096x16384_b4_loguniform": dict(N1=4096, N2=1 << 14, p=64, b=4, gen="loguniform", seed=5),
}


def make(gen: str, N: int, seed: int) -> np.ndarray:
    return {"uniform": uniform, "normal": normal, "loguniform": loguniform}[gen](N, seed)
