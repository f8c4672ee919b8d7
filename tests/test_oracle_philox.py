"""Pins of the oracle's Philox4x32-10 and of the draw -> uniform mapping."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(oracle_mod, ctr, key, expect):
    out = oracle_mod.philox4x32_10(ctr, key)
    assert [int(x) for x in out] == expect


@pytest.fixture(scope="module")
def rocrand_ref():
    """rocRAND's header Philox, built on the host as a second implementation."""
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(hdr) or shutil.which("g++") is None:
        pytest.skip("rocRAND headers or g++ not available")
    d = tempfile.mkdtemp(prefix="rr_")
    so = os.path.join(d, "rr.so")
    subprocess.run(["g++", "-O1", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", "-o", so,
                    os.path.join(HERE, "rocrand_philox_ref.cpp")], check=True)
    L = ctypes.CDLL(so)
    L.rocrand_philox_ref.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int]
    return L


def test_philox_matches_rocrand(oracle_mod, rocrand_ref):
    rng = np.random.default_rng(20260)
    n = 2000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:, 1] >>= 2  # rocRAND's 64-bit offset = 4 * (ctr1:ctr0) must not wrap
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    out = np.zeros((n, 4), dtype=np.uint32)
    P = ctypes.c_void_p
    rocrand_ref.rocrand_philox_ref(ctr.ctypes.data_as(P), key.ctypes.data_as(P),
                                   out.ctypes.data_as(P), n)
    ref = np.array([oracle_mod.philox4x32_10(ctr[k], key[k]) for k in range(n)])
    assert np.array_equal(ref, out)


def test_uniform_is_exact_24bit_and_below_one(oracle_mod):
    # u = (r >> 8) * 2^-24 is exact: u * 2^24 is an integer in [0, 2^24 - 1]
    for seed in (0, 1, 2**40 + 7):
        for (t, c, i) in [(0, 0, 0), (3, 5, 7), (199, 4095, 199999), (1, 2, 3)]:
            u = oracle_mod.uniform(seed, t, c, i)
            m = u * 2.0**24
            assert m == int(m) and 0 <= m <= 2**24 - 1


def test_uniform_counter_layout(oracle_mod):
    """Reading: gene i of chromosome c at generation t takes word i%4 of
    Philox(ctr={i/4, c, t, 0}, key={seed lo, seed hi})."""
    seed = 0x0123456789ABCDEF
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for (t, c, k) in [(0, 0, 0), (7, 3, 11), (1000, 1023, 2499), (5, 0, 1)]:
        words = oracle_mod.philox4x32_10([k, c, t, 0], key)
        for j in range(4):
            u = oracle_mod.uniform(seed, t, c, 4 * k + j)
            assert u * 2.0**24 == int(words[j]) >> 8


def test_uniform_streams_differ(oracle_mod):
    base = [oracle_mod.uniform(9, 4, 2, i) for i in range(64)]
    assert len(set(base)) > 60
    assert base != [oracle_mod.uniform(9, 5, 2, i) for i in range(64)]   # generation
    assert base != [oracle_mod.uniform(9, 4, 3, i) for i in range(64)]   # chromosome
    assert base != [oracle_mod.uniform(10, 4, 2, i) for i in range(64)]  # seed


def test_uniform_mean_and_range(oracle_mod):
    u = np.array([oracle_mod.uniform(3, 0, c, i) for c in range(8) for i in range(1000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    # mean of U[0,1): 0.5 +- 6 sigma, sigma = sqrt(1/12/n)
    assert abs(u.mean() - 0.5) < 6 * np.sqrt(1 / 12 / u.size)
