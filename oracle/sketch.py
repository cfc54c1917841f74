"""Subspace-embedding sketches Theta (oracle side, test infrastructure).

Section 2.1.1 of the paper draws Theta in R^{s x n} as a subsampled randomized
Hadamard transform (s rows sampled uniformly from the Walsh-Hadamard transform
times a diagonal of Rademacher signs) and names sparse sign matrices as an
alternative.  The paper does not fix the normalisation, the padding or the
sampling rule; this build reads them as follows (the GPU library implements
the same written definition independently):

SRHT      n' = 2^ceil(log2 n), x zero-padded to n';
          Theta x = s^{-1/2} (H_{n'} D x)[P]
          H[a, b] = (-1)^popcount(a & b)  (unnormalised Sylvester order),
          D[i]    = -1 if bit 63 of value(seed, 1, i) is set else +1,
          P       = s distinct rows of [0, n') by Floyd's sampling: for
                    t = 0..s-1, j = n' - s + t, q = floor(value(seed, 2, t) (j+1) / 2^64);
                    take q unless already taken, else take j.
          E ||Theta x||^2 = ||x||^2.
sparse    column i has zeta distinct nonzero rows, by Floyd's sampling over
sign      [0, s): for t = 0..zeta-1, j = s - zeta + t,
          w = value(seed, 3, i*ceil(zeta/2) + floor(t/2)),
          h = high 32 bits of w for even t, low 32 bits for odd t,
          q = floor(h (j+1) / 2^32); take q unless already taken, else j.
          Entry (row_t, i) = +-1/sqrt(zeta), negative iff bit t of
          value(seed, 4, i) is set.  E ||Theta x||^2 = ||x||^2.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import rng


def next_pow2(n: int) -> int:
    return 1 << max(0, (n - 1).bit_length())


# ----------------------------------------------------------------------------- SRHT
def srht_signs(n: int, seed: int) -> np.ndarray:
    v = rng.values(seed, rng.STREAM_SRHT_SIGNS, np.arange(n))
    return np.where((v >> np.uint64(63)) != 0, -1.0, 1.0)


def srht_rows(n: int, s: int, seed: int) -> np.ndarray:
    npad = next_pow2(n)
    if not 0 < s <= npad:
        raise ValueError("need 0 < s <= padded length")
    chosen, seen = [], set()
    for t in range(s):
        j = npad - s + t
        q = (rng.value(seed, rng.STREAM_SRHT_ROWS, t) * (j + 1)) >> 64
        pick = j if q in seen else q
        seen.add(pick)
        chosen.append(pick)
    return np.array(chosen, dtype=np.int64)


def fwht(x: np.ndarray) -> np.ndarray:
    """Unnormalised Walsh-Hadamard transform along axis 0 (Sylvester order), length 2^p."""
    y = np.array(x, dtype=np.float64, copy=True)
    n = y.shape[0]
    if n & (n - 1):
        raise ValueError("length must be a power of two")
    tail = y.shape[1:]
    h = 1
    while h < n:
        z = y.reshape((n // (2 * h), 2, h) + tail)
        a = z[:, 0].copy()
        b = z[:, 1]
        z[:, 0] = a + b
        z[:, 1] = a - b
        h *= 2
    return y


def srht_apply(X: np.ndarray, s: int, seed: int) -> np.ndarray:
    """Theta X for a vector or an n x c matrix X."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    npad = next_pow2(n)
    d = srht_signs(n, seed)
    Y = np.zeros((npad,) + X.shape[1:])
    Y[:n] = (d.reshape((n,) + (1,) * (X.ndim - 1))) * X
    return fwht(Y)[srht_rows(n, s, seed)] / math.sqrt(s)


def srht_dense(n: int, s: int, seed: int) -> np.ndarray:
    """Theta as a dense s x n matrix, from the entry formula (small n only)."""
    rows = srht_rows(n, s, seed)
    d = srht_signs(n, seed)
    cols = np.arange(n)
    pc = np.vectorize(lambda v: bin(int(v)).count("1") & 1)
    H = 1.0 - 2.0 * pc(rows[:, None] & cols[None, :])
    return H * d[None, :] / math.sqrt(s)


# ----------------------------------------------------------------------------- sparse sign
def sparse_sign_pattern(n: int, s: int, zeta: int, seed: int):
    """(rows[n, zeta], signs[n, zeta]) of the sparse-sign Theta."""
    if not 1 <= zeta <= min(s, 64):
        raise ValueError("need 1 <= zeta <= min(s, 64)")
    half = (zeta + 1) // 2
    cols = np.arange(n, dtype=np.uint64)
    rows = np.zeros((n, zeta), dtype=np.int64)
    for t in range(zeta):
        j = s - zeta + t
        w = rng.values(seed, rng.STREAM_SPARSE_ROWS, cols * np.uint64(half) + np.uint64(t // 2))
        h = (w >> np.uint64(32)) if t % 2 == 0 else (w & np.uint64(0xFFFFFFFF))
        q = ((h * np.uint64(j + 1)) >> np.uint64(32)).astype(np.int64)
        taken = (rows[:, :t] == q[:, None]).any(axis=1) if t else np.zeros(n, dtype=bool)
        rows[:, t] = np.where(taken, j, q)
    sbits = rng.values(seed, rng.STREAM_SPARSE_SIGNS, cols)
    signs = np.empty((n, zeta))
    for t in range(zeta):
        signs[:, t] = np.where(((sbits >> np.uint64(t)) & np.uint64(1)) != 0, -1.0, 1.0)
    return rows, signs


def sparse_sign_matrix(n: int, s: int, zeta: int, seed: int) -> sp.csc_matrix:
    rows, signs = sparse_sign_pattern(n, s, zeta, seed)
    colidx = np.repeat(np.arange(n), zeta)
    return sp.csc_matrix((signs.ravel() / math.sqrt(zeta), (rows.ravel(), colidx)), shape=(s, n))


# ----------------------------------------------------------------------------- dispatch
class Sketch:
    """Theta for one (kind, n, s, zeta, seed); ``apply`` maps n x c to s x c."""

    def __init__(self, kind: str, n: int, s: int, seed: int, zeta: int = 8):
        self.kind, self.n, self.s, self.seed, self.zeta = kind, n, s, seed, zeta
        if kind == "sparse_sign":
            self._M = sparse_sign_matrix(n, s, zeta, seed)
        elif kind != "srht":
            raise ValueError(kind)

    def apply(self, X: np.ndarray) -> np.ndarray:
        if self.kind == "srht":
            return srht_apply(X, self.s, self.seed)
        return np.asarray(self._M @ X)

    def dense(self) -> np.ndarray:
        if self.kind == "srht":
            return srht_dense(self.n, self.s, self.seed)
        return self._M.toarray()
