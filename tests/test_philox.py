"""Statistical pins of the counter-based generator the oracle draws from
(Philox4x32-10, Salmon et al., SC'11).  Bit-level agreement with the GPU
library's own implementation is a GPU parity test."""
import numpy as np

import oracle


def _block(n, key=(7, 9), word3=0):
    out = np.zeros((n, 4), dtype=np.uint64)
    for c in range(n):
        out[c] = oracle.philox4x32_10([c, 0, 0, word3], list(key))
    return out


def test_uniformity_and_moments():
    w = _block(5000).ravel()
    u = (w.astype(np.float64) + 0.5) / 2.0 ** 32
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / u.size)
    assert abs(u.var() - 1 / 12) < 0.003
    hist, _ = np.histogram(u, bins=32, range=(0, 1))
    expected = u.size / 32
    chi2 = ((hist - expected) ** 2 / expected).sum()
    assert chi2 < 70          # 31 degrees of freedom; p ~ 1e-4


def test_bits_are_balanced():
    w = _block(4000).ravel()
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint64)) & 1).astype(np.float64)
    frac = bits.mean(axis=0)
    assert np.all(np.abs(frac - 0.5) < 5 * np.sqrt(0.25 / w.size))


def test_counter_and_key_sensitivity():
    a = oracle.philox4x32_10([1, 2, 3, 4], [5, 6])
    for ctr, key in [([1, 2, 3, 5], [5, 6]), ([0, 2, 3, 4], [5, 6]), ([1, 2, 3, 4], [5, 7])]:
        b = oracle.philox4x32_10(ctr, key)
        flipped = sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b))
        assert 32 < flipped < 96     # avalanche: about half of the 128 bits change


def test_distinct_counters_distinct_outputs():
    w = _block(3000)
    rows = {tuple(r) for r in w.tolist()}
    assert len(rows) == w.shape[0]


def test_adjacent_outputs_uncorrelated():
    w = _block(5000)
    u = (w.astype(np.float64) + 0.5) / 2.0 ** 32
    for a, b in [(0, 1), (1, 2), (2, 3)]:
        assert abs(np.corrcoef(u[:, a], u[:, b])[0, 1]) < 0.05
    assert abs(np.corrcoef(u[:-1, 0], u[1:, 0])[0, 1]) < 0.05
