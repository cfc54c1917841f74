"""SplitMix64 counter streams (oracle side, test infrastructure).

SplitMix64 is the generator of Steele, Lea & Flood (OOPSLA 2014) in the form
published by S. Vigna: the state advances by the golden gamma
0x9E3779B97F4A7C15 and each output is the state passed through the
"variant 13" 64-bit finaliser.  The paper leaves the random source of the
sketch unspecified ("draw sketch matrix Theta", Algorithm 1); this build fixes
it as a counter-based stream so that the oracle and the GPU library can
generate the same Theta independently:

    out(seed, i)          = finalise(seed + (i + 1) * gamma)      (mod 2^64)
    value(seed, stream, i) = out(out(seed, stream), i)

Pinned by the published first outputs of SplitMix64 seeded with 0.
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1

STREAM_SRHT_SIGNS = 1
STREAM_SRHT_ROWS = 2
STREAM_SPARSE_ROWS = 3
STREAM_SPARSE_SIGNS = 4


def finalise(z: int) -> int:
    z &= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def out(seed: int, i: int) -> int:
    return finalise((seed + (i + 1) * GAMMA) & _M64)


def value(seed: int, stream: int, i: int) -> int:
    return out(out(seed, stream), i)


def _finalise_vec(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def values(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Vectorised value(seed, stream, i) for an integer index array."""
    key = np.uint64(out(seed, stream))
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = key + (idx + np.uint64(1)) * np.uint64(GAMMA)
    return _finalise_vec(z)
