"""Method-internal randomness of the oracle (test infrastructure).

Algorithm 2 samples S > R rows uniformly, and Sec. 4.1 interpolates from a random ~10%
subset of the data; the paper names no generator, no replacement rule and no order.
Reading taken: draws are without replacement, returned sorted ascending, and come from a
partial Fisher-Yates shuffle driven by SplitMix64.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014; the 64-bit finaliser constants are Stafford's "Mix13"): the state advances by
the golden-ratio increment 0x9E3779B97F4A7C15 and each output is the state passed through
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)
The i-th output (i = 0, 1, ...) of a stream started at state s is mix(s + (i+1)*gamma).

A bounded draw in [0, n) takes the high 64 bits of the 128-bit product r * n.
Stream seeds: state = seed * 256 + stream; stream 1 is the interpolation subset, stream 2
the least-squares rows.
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

STREAM_INTERP = 1
STREAM_LS = 2


def stream_state(seed: int, stream: int) -> int:
    return (int(seed) * 256 + int(stream)) & MASK64


def splitmix64(state: int, count: int) -> np.ndarray:
    """The first ``count`` outputs of a SplitMix64 stream started at ``state`` (uint64)."""
    i = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(state) + i * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        z = z ^ (z >> np.uint64(31))
    return z


def bounded(r: np.ndarray, n: np.ndarray) -> np.ndarray:
    """floor(r * n / 2^64) for uint64 r and n < 2^32, computed exactly in 64-bit pieces."""
    r = r.astype(np.uint64)
    n = n.astype(np.uint64)
    hi = r >> np.uint64(32)
    lo = r & np.uint64(0xFFFFFFFF)
    with np.errstate(over="ignore"):
        t = hi * n + ((lo * n) >> np.uint64(32))
    return t >> np.uint64(32)


def sample_without_replacement(seed: int, stream: int, n: int, m: int) -> np.ndarray:
    """m distinct indices of [0, n), sorted ascending (int64)."""
    if not (0 <= m <= n):
        raise ValueError("need 0 <= m <= n")
    if n >= (1 << 32):
        raise ValueError("n must be below 2^32")
    r = splitmix64(stream_state(seed, stream), m)
    i = np.arange(m, dtype=np.uint64)
    j = (i + bounded(r, np.uint64(n) - i)).astype(np.int64)
    a = np.arange(n, dtype=np.int64)
    for t in range(m):                      # the shuffle itself is sequential
        jt = j[t]
        a[t], a[jt] = a[jt], a[t]
    return np.sort(a[:m])


STREAM_BATCH = 3


def batch_indices(seed: int, step: int, batch: int, n: int) -> np.ndarray:
    """Minibatch of the corrector's training step `step` (0-based): `batch` indices of [0, n)
    drawn with replacement.  Index i is the bounded draw of SplitMix64 output number
    step * batch + i of the stream seed * 256 + 3 (counter form, so any step can be drawn
    without the previous ones)."""
    state = stream_state(seed, STREAM_BATCH)
    k = np.arange(step * batch, (step + 1) * batch, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(state) + (k + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        z = z ^ (z >> np.uint64(31))
    return bounded(z, np.uint64(n)).astype(np.int64)
