"""Pins of the counter-based generator the oracle draws from (Philox4x32-10,
Salmon et al., SC'11): the published known-answer values, bitwise agreement
with an implementation written by others (rocRAND's engine header, compiled
for the host from the ROCm image's source), and statistical checks.
Bit-level agreement with the GPU library's own implementation is a GPU parity
test."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
REF_SRC = os.path.join(HERE, "rocrand_ref", "philox_ref.cpp")
REF_LIB = os.path.join(HERE, "rocrand_ref", "libphilox_ref.so")
ROCM_INC = "/opt/rocm/include"


def _rocrand_ref():
    """rocRAND's Philox4x32-10 engine built for the host (g++), or None without the header"""
    if not os.path.exists(os.path.join(ROCM_INC, "rocrand", "rocrand_philox4x32_10.h")) or not shutil.which("g++"):
        return None
    if not os.path.exists(REF_LIB) or os.path.getmtime(REF_LIB) < os.path.getmtime(REF_SRC):
        subprocess.check_call(["g++", "-O1", "-fPIC", "-shared", "-std=c++17", "-D__HIP_PLATFORM_AMD__",
                               "-I" + ROCM_INC, "-o", REF_LIB + ".tmp", REF_SRC])
        os.replace(REF_LIB + ".tmp", REF_LIB)
    lib = C.CDLL(REF_LIB)
    lib.ref_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]
    lib.ref_philox4x32_10.restype = None
    return lib


def _oracle_many(ctr, key):
    return np.array([oracle.philox4x32_10(list(c), list(k)) for c, k in zip(ctr.tolist(), key.tolist())],
                    dtype=np.uint32)


def test_known_answers():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert [int(x) for x in oracle.philox4x32_10(v[0:4], v[4:6])] == v[6:10]


def test_bitwise_equal_to_rocrand_engine():
    lib = _rocrand_ref()
    if lib is None:
        pytest.skip("rocRAND headers or g++ not available")
    rng = np.random.default_rng(20240611)
    # edge words (0, 1, 2^31, 2^32 - 1) in every position, then random counters and keys,
    # and the counter layouts the method uses: (id, id, step low, step high | tag << 28)
    edge = np.array([0, 1, 0x80000000, 0xFFFFFFFF], dtype=np.uint32)
    ctr = [np.array(np.meshgrid(edge, edge, edge, edge)).reshape(4, -1).T]
    key = [np.tile(edge[[3, 0]], (ctr[0].shape[0], 1))]
    ctr.append(rng.integers(0, 2 ** 32, size=(3000, 4), dtype=np.uint64).astype(np.uint32))
    key.append(rng.integers(0, 2 ** 32, size=(3000, 2), dtype=np.uint64).astype(np.uint32))
    ids = rng.integers(0, 1 << 26, size=(2000, 2))
    steps = rng.integers(0, 1 << 40, size=2000, dtype=np.int64)
    tags = rng.integers(0, 4, size=2000)
    c = np.stack([ids.min(1), ids.max(1), steps & 0xFFFFFFFF, ((steps >> 32) & 0x0FFFFFFF) | (tags << 28)], 1)
    ctr.append(c.astype(np.uint32))
    key.append(np.tile(np.array([3, 0], dtype=np.uint32), (2000, 1)))
    ctr = np.ascontiguousarray(np.concatenate(ctr))
    key = np.ascontiguousarray(np.concatenate(key))
    out = np.zeros_like(ctr)
    lib.ref_philox4x32_10(ctr.ctypes.data, key.ctypes.data, out.ctypes.data, ctr.shape[0])
    np.testing.assert_array_equal(_oracle_many(ctr, key), out)


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
