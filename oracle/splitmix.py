"""SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), evaluated as a counter-based generator.

The k-th output (k = 0, 1, ...) of the generator seeded with s is
mix(s + (k+1) * 0x9E3779B97F4A7C15 mod 2^64), where mix is the published
finalizer.  A double on [0,1) takes the top 53 bits; the Lanczos start vector
entry is 2u - 1 before normalisation.  All steps are exact, so any correct
implementation reproduces the same doubles bit for bit.
"""
import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1


def splitmix64_mix(z: int) -> int:
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def splitmix64_outputs(seed: int, count: int):
    """First `count` outputs of the sequential generator (plain Python ints)."""
    state = seed & MASK
    out = []
    for _ in range(count):
        state = (state + GAMMA) & MASK
        out.append(splitmix64_mix(state))
    return out


def start_vector(seed: int, D: int, chunk: int = 1 << 22) -> np.ndarray:
    """Unnormalised start vector v[r] = 2 u_r - 1, u_r from output r of SplitMix64(seed)."""
    v = np.empty(D, dtype=np.float64)
    with np.errstate(over="ignore"):
        for lo in range(0, D, chunk):
            hi = min(D, lo + chunk)
            k = np.arange(lo + 1, hi + 1, dtype=np.uint64)
            z = np.uint64(seed & MASK) + k * np.uint64(GAMMA)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            z = z ^ (z >> np.uint64(31))
            u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
            v[lo:hi] = 2.0 * u - 1.0
    return v
