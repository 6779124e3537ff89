"""Sparse-sign sketching operator S (oracle side) -- test infrastructure only.

S is an s x N matrix that acts as an epsilon-subspace embedding (Section 3,
eq. (3.1)).  This build uses the sparse-sign family: every column holds
exactly zeta nonzeros of value +-1/sqrt(zeta), one in each of zeta row blocks
of height s/zeta (the block construction of Kane and Nelson, so the rows of a
column are distinct without rejection).

The random choices are a fixed function of (seed, column, block) so that the
GPU path, which regenerates S on the fly, can draw the identical operator
from its own implementation of the same published generator:

* counter  c(n, g) = n*G + g + 1, with G = ceil(zeta/4) hash words per column;
* key      = seed + 0x9E3779B97F4A7C15 * c   (mod 2^64);
* h        = SplitMix64 output mixer of key (Steele, Lea and Flood, OOPSLA
  2014; the mixer constants are Stafford's "Mix13");
* block b = 4g + q takes the 16-bit field u = (h >> 16q) & 0xFFFF;
  row  = b*(s/zeta) + (((u >> 1) * (s/zeta)) >> 15),
  sign = -1 if (u & 1) else +1.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def sketch_pattern(N: int, s: int, zeta: int, seed: int):
    """Rows (N x zeta, int64) and signs (N x zeta, +-1.0) of S's nonzeros."""
    if zeta < 1 or s % zeta != 0:
        raise ValueError("s must be a positive multiple of zeta")
    bsz = s // zeta
    G = (zeta + 3) // 4
    n = np.arange(N, dtype=np.uint64)
    rows = np.empty((N, zeta), dtype=np.int64)
    signs = np.empty((N, zeta), dtype=np.float64)
    with np.errstate(over="ignore"):
        for g in range(G):
            ctr = n * np.uint64(G) + np.uint64(g + 1)
            key = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + _GAMMA * ctr
            h = splitmix64_mix(key)
            for q in range(4):
                b = 4 * g + q
                if b >= zeta:
                    break
                u = (h >> np.uint64(16 * q)) & np.uint64(0xFFFF)
                off = ((u >> np.uint64(1)) * np.uint64(bsz)) >> np.uint64(15)
                rows[:, b] = b * bsz + off.astype(np.int64)
                signs[:, b] = np.where((u & np.uint64(1)) == 1, -1.0, 1.0)
    return rows, signs


def sketch_operator(N: int, s: int, zeta: int, seed: int) -> sp.csr_matrix:
    """Explicit s x N sparse-sign matrix (float64, CSR)."""
    rows, signs = sketch_pattern(N, s, zeta, seed)
    cols = np.repeat(np.arange(N, dtype=np.int64), zeta)
    vals = signs.reshape(-1) / np.sqrt(zeta)
    return sp.csr_matrix((vals, (rows.reshape(-1), cols)), shape=(s, N))
