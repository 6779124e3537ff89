"""Subsampled randomised DCT sketch S = sqrt(N/s) P F E (oracle side) -- test
infrastructure only.

The paper's own sketching operator (Section 6): E is an N x N diagonal of
random signs, F the N-point discrete cosine transform, and P selects s of
the rows of F E at random (the subsampled randomised trigonometric
transform).  Readings taken here (the paper states neither):

* F is the orthonormal DCT-II: F[k, n] = c_k cos(pi k (2n + 1) / (2N)),
  c_0 = sqrt(1/N), c_k = sqrt(2/N);
* the scale sqrt(N/s) makes S an isometry in expectation (E ||S x||^2 =
  ||x||^2), so that the embedding bound of eq. (3.1) holds with a small eps.

The random choices are fixed functions of the seed, so that the GPU path can
draw the same operator from its own implementation of the same published
generator (the SplitMix64 output mixer, as for the sparse-sign sketch):

* sign of row n: -1 if bit 0 of mix64(seed ^ SIGN_SALT + GAMMA (n + 1)) is
  set, else +1;
* rows kept: the s indices n in [0, N) with the smallest keys
  mix64(seed ^ ROW_SALT + GAMMA (n + 1)) (ties by index), in increasing n.
"""

from __future__ import annotations

import numpy as np
import scipy.fft

from .sketch import splitmix64_mix

GAMMA = np.uint64(0x9E3779B97F4A7C15)
SIGN_SALT = 0x5851F42D4C957F2D
ROW_SALT = 0x14057B7EF767814F


def _keys(N: int, seed: int, salt: int) -> np.ndarray:
    base = np.uint64((seed ^ salt) & 0xFFFFFFFFFFFFFFFF)
    n = np.arange(1, N + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return splitmix64_mix(base + GAMMA * n)


def srdct_signs(N: int, seed: int) -> np.ndarray:
    """Diagonal of E: +-1.0 per row."""
    return np.where((_keys(N, seed, SIGN_SALT) & np.uint64(1)) == 1, -1.0, 1.0)


def srdct_rows(N: int, s: int, seed: int) -> np.ndarray:
    """The s DCT frequencies kept by P, increasing."""
    if not 1 <= s <= N:
        raise ValueError("need 1 <= s <= N")
    k = _keys(N, seed, ROW_SALT)
    order = np.lexsort((np.arange(N), k))  # by key, then index
    return np.sort(order[:s])


class SRDCT:
    """The operator S (s x N).  ``S @ X`` for a vector or an N x c block
    applies E, the orthonormal DCT-II along the rows (scipy.fft.dct), keeps
    the rows P and scales by sqrt(N/s)."""

    def __init__(self, N: int, s: int, seed: int):
        self.N, self.s, self.seed = N, s, seed
        self.shape = (s, N)
        self.signs = srdct_signs(N, seed)
        self.rows = srdct_rows(N, s, seed)
        self.scale = np.sqrt(N / s)

    def __matmul__(self, X):
        X = np.asarray(X)
        one = X.ndim == 1
        Y = X.reshape(self.N, -1) * self.signs[:, None]
        if np.iscomplexobj(Y):
            F = (scipy.fft.dct(Y.real, type=2, norm="ortho", axis=0)
                 + 1j * scipy.fft.dct(Y.imag, type=2, norm="ortho", axis=0))
        else:
            F = scipy.fft.dct(Y, type=2, norm="ortho", axis=0)
        out = self.scale * F[self.rows]
        return out[:, 0] if one else out

    def toarray(self) -> np.ndarray:
        """Explicit s x N matrix (small N only)."""
        return self @ np.eye(self.N)
