"""Pins of the oracle's sketching operator (Section 3, eq. (3.1))."""

import os

import numpy as np

from oracle.sketch import sketch_operator, sketch_pattern, splitmix64_mix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vector():
    vals = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    gamma = 0x9E3779B97F4A7C15
    state = 1234567
    keys = []
    for _ in range(5):
        state = (state + gamma) % 2 ** 64
        keys.append(state)
    out = splitmix64_mix(np.array(keys, dtype=np.uint64))
    assert [int(v) for v in out] == vals


def _mix_py(z):
    """Pure-Python big-int transcription of the mixer (independent of numpy)."""
    M = 2 ** 64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) % M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) % M
    return z ^ (z >> 31)


def test_pattern_against_bigint_definition():
    N, s, zeta, seed = 37, 120, 8, 42
    rows, signs = sketch_pattern(N, s, zeta, seed)
    bsz = s // zeta
    for n in range(N):
        for b in range(zeta):
            g, q = divmod(b, 4)
            key = (seed + 0x9E3779B97F4A7C15 * (n * 2 + g + 1)) % 2 ** 64
            u = (_mix_py(key) >> (16 * q)) & 0xFFFF
            assert rows[n, b] == b * bsz + (((u >> 1) * bsz) >> 15)
            assert signs[n, b] == (-1.0 if u & 1 else 1.0)


def test_structure_one_nonzero_per_block():
    N, s, zeta = 5000, 240, 8
    S = sketch_operator(N, s, zeta, 7).tocsc()
    bsz = s // zeta
    assert S.nnz == N * zeta
    for n in range(0, N, 97):
        col = S[:, n]
        r = np.sort(col.indices)
        assert r.shape[0] == zeta
        np.testing.assert_array_equal(r // bsz, np.arange(zeta))
        np.testing.assert_allclose(np.abs(col.data), 1 / np.sqrt(zeta))
    # rows roughly balanced, signs roughly balanced
    counts = np.bincount(S.tocoo().row, minlength=s)
    assert counts.min() > 0.7 * N * zeta / s and counts.max() < 1.3 * N * zeta / s
    assert abs(np.mean(np.sign(S.data))) < 0.05


def test_norm_preserved_in_expectation_and_embedding():
    N, s, zeta = 4000, 160, 8
    rng = np.random.default_rng(0)
    v = rng.standard_normal(N)
    ratios = [np.linalg.norm(sketch_operator(N, s, zeta, sd) @ v) ** 2 / np.dot(v, v)
              for sd in range(30)]
    assert abs(np.mean(ratios) - 1.0) < 0.05
    # epsilon of the embedding of a 20-dimensional subspace stays well below 1
    Q, _ = np.linalg.qr(rng.standard_normal((N, 20)))
    sv = np.linalg.svd(sketch_operator(N, s, zeta, 3) @ Q, compute_uv=False)
    eps = max(sv[0] ** 2 - 1, 1 - sv[-1] ** 2)
    assert eps < 0.8


def test_seed_and_shape_dependence():
    r1, _ = sketch_pattern(100, 120, 8, 1)
    r2, _ = sketch_pattern(100, 120, 8, 2)
    assert np.mean(r1 == r2) < 0.2
    # zeta not a multiple of four still fills every block
    r3, s3 = sketch_pattern(50, 60, 6, 5)
    np.testing.assert_array_equal(r3 // 10, np.tile(np.arange(6), (50, 1)))
