"""SplitMix64 (Steele, Lea, Flood 2014; Vigna's reference formulation).

The Arnoldi start vector is the one random draw inside the setup; the paper
leaves it unspecified (Sec. 2.3), so both implementations derive it from the
published SplitMix64 sequence:

    state_i = seed + (i + 1) * 0x9E3779B97F4A7C15        (mod 2^64)
    z = state_i
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    out_i = z ^ (z >> 31)

and v0[i] = 2 * u_i - 1 with u_i = (out_i >> 11) * 2^-53.
"""
import numpy as np

_M = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64_outputs(seed, count):
    """First `count` outputs of SplitMix64 started from `seed` (Python ints)."""
    out = []
    for i in range(count):
        z = (seed + (i + 1) * GAMMA) & _M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M
        out.append(z ^ (z >> 31))
    return out


def start_vector(seed, n):
    """Unnormalised Arnoldi start vector v0 of length n (float64)."""
    seed = int(seed) & _M
    z = (np.uint64(seed) + (np.arange(1, n + 1, dtype=np.uint64) *
                            np.uint64(GAMMA)))
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0
