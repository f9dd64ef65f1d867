"""Pins of the oracle's core engine (Philox4x32-10, Salmon et al. SC'11).

The engine is the paper's "core engine RNG" slot (Sec. 2.2); the paper does
not fix one.  The oracle's implementation is checked against an independent
one (rocRAND's host-callable Philox4x32-10 engine, compiled from its header
here), and against structural properties any correct Philox must have.
"""
import os
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROCRAND_INC = "/opt/rocm/include"


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    if not os.path.exists(os.path.join(ROCRAND_INC, "rocrand", "rocrand_philox4x32_10.h")):
        pytest.skip("rocRAND headers not installed")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_ref")
    subprocess.check_call(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", ROCRAND_INC,
                           os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe])

    def run(cases):
        inp = "\n".join(" ".join(str(int(v)) for v in c) for c in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return np.array([[int(x) for x in ln.split()] for ln in out.strip().splitlines()],
                        dtype=np.uint64)
    return run


def test_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(11)
    cases = []
    edges = [0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF]
    for e in edges:
        cases.append([e, 0, 0, 0, 0, 0])
        cases.append([0, 0, e, 0, 0, 0])
        cases.append([0, 0, 0, e, 0, 0])
        cases.append([0, 0, 0, 0, e, 0])
        cases.append([0, 0, 0, 0, 0, e])
        cases.append([e, e & 0x3FFFFFFF, e, e, e, e])
    for _ in range(1500):
        c = rng.integers(0, 2**32, size=6, dtype=np.uint64)
        c[1] &= 0x3FFFFFFF  # the reference helper's offset argument must not overflow
        cases.append(list(c))
    ref = rocrand_ref(cases)
    got = np.array([oracle.philox4x32(c[:4], c[4:]) for c in cases], dtype=np.uint64)
    assert np.array_equal(got, ref)


def test_zero_rounds_is_identity():
    for ctr in ([0, 0, 0, 0], [1, 2, 3, 4], [0xFFFFFFFF] * 4):
        assert list(oracle.philox4x32(ctr, [5, 6], rounds=0)) == ctr


def test_one_round_by_hand():
    M0, M1 = 0xD2511F53, 0xCD9E8D57
    rng = np.random.default_rng(3)
    for _ in range(200):
        c = [int(x) for x in rng.integers(0, 2**32, 4, dtype=np.uint64)]
        k = [int(x) for x in rng.integers(0, 2**32, 2, dtype=np.uint64)]
        p0, p1 = M0 * c[0], M1 * c[2]
        want = [((p1 >> 32) ^ c[1] ^ k[0]) & 0xFFFFFFFF, p1 & 0xFFFFFFFF,
                ((p0 >> 32) ^ c[3] ^ k[1]) & 0xFFFFFFFF, p0 & 0xFFFFFFFF]
        assert list(oracle.philox4x32(c, k, rounds=1)) == want


def _popcount(a):
    a = a.astype(np.uint64)
    return np.array([bin(int(x)).count("1") for x in a])


def test_avalanche():
    rng = np.random.default_rng(5)
    fr = []
    for _ in range(40):
        c = [int(x) for x in rng.integers(0, 2**32, 4, dtype=np.uint64)]
        k = [int(x) for x in rng.integers(0, 2**32, 2, dtype=np.uint64)]
        base = oracle.philox4x32(c, k)
        for bit in range(128):
            cc = list(c)
            cc[bit // 32] ^= 1 << (bit % 32)
            fr.append(_popcount(base ^ oracle.philox4x32(cc, k)).sum() / 128.0)
    fr = np.array(fr)
    assert abs(fr.mean() - 0.5) < 0.01
    assert fr.min() > 0.25 and fr.max() < 0.75


def test_byte_uniformity():
    w = oracle.words(2024, 3, 0, 0, 1 << 16)
    bytes_ = w.view(np.uint8)
    counts = np.bincount(bytes_, minlength=256)
    chi2, p = stats.chisquare(counts)
    assert p > 1e-4


def test_streams_are_distinct():
    a = oracle.words(1, 0, 0, 0, 64)
    assert not np.array_equal(a, oracle.words(1, 1, 0, 0, 64))  # unit
    assert not np.array_equal(a, oracle.words(1, 0, 1, 0, 64))  # kind
    assert not np.array_equal(a, oracle.words(2, 0, 0, 0, 64))  # seed low
    assert not np.array_equal(a, oracle.words(1 + (1 << 32), 0, 0, 0, 64))  # seed high
    # block index high word is part of the counter
    assert not np.array_equal(oracle.words(1, 0, 0, 5, 1), oracle.words(1, 0, 0, 5 + (1 << 32), 1))
