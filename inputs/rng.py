"""Counter-based SplitMix64 streams (Steele, Lea and Flood, OOPSLA 2014).

A draw is a pure function of (seed, stream, counter):

    key    = mix64(seed XOR (stream * 0xD1B54A32D192ED03))
    draw_k = mix64(key + (k + 1) * 0x9E3779B97F4A7C15)

where mix64 is the SplitMix64 output finaliser (Stafford's "variant 13").
Because every draw is addressed by its counter, generation can be done in
any order or in chunks and still give identical values.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_STREAM_MUL = np.uint64(0xD1B54A32D192ED03)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_TWO_M53 = 2.0 ** -53


def splitmix64(z):
    """SplitMix64 finaliser applied element-wise to a uint64 array."""
    z = np.asarray(z, dtype=np.uint64).copy()
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def _key(seed, stream):
    s = np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    st = np.array([stream & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    return splitmix64(s ^ (st * _STREAM_MUL))[0]


def u64_stream(seed, stream, counters):
    """Raw 64-bit draws for the given counter array."""
    c = np.asarray(counters, dtype=np.uint64)
    return splitmix64(_key(seed, stream) + (c + np.uint64(1)) * _GAMMA)


def uniform(seed, stream, counters):
    """Doubles in [0, 1): the top 53 bits of each draw times 2**-53."""
    return (u64_stream(seed, stream, counters) >> np.uint64(11)).astype(np.float64) * _TWO_M53


def normal(seed, stream, counters):
    """Standard normal draws by Box-Muller; draw i uses counters 2i and 2i+1."""
    c = np.asarray(counters, dtype=np.uint64)
    u1 = 1.0 - uniform(seed, stream, c * np.uint64(2))          # (0, 1]
    u2 = uniform(seed, stream, c * np.uint64(2) + np.uint64(1))  # [0, 1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
