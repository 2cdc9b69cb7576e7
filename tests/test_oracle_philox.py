"""Pins for the oracle's Philox4x32-10 and the Bernoulli selection of eq. (2).

The generator is checked against rocRAND's open-source Philox header, compiled
here as a host program (an implementation independent of the oracle), and the
selection is checked statistically: the sampled fraction is Binomial(n, p),
two draws overlap with rate p^2, and p = 1 selects every coordinate.
"""

import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle.csc import sample_threshold

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def philox_ref(tmp_path_factory):
    gxx = shutil.which("g++")
    inc = "/opt/rocm/include"
    if gxx is None or not os.path.exists(os.path.join(inc, "rocrand", "rocrand_philox4x32_10.h")):
        pytest.skip("host C++ compiler or rocRAND header not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run(
        [gxx, "-O1", "-D__HIP_PLATFORM_AMD__", "-I" + inc, os.path.join(HERE, "philox_ref_host.cpp"), "-o", exe],
        check=True,
        capture_output=True,
    )

    def run(rows):
        text = "".join("%x %x %x %x %x %x\n" % tuple(int(v) for v in row) for row in rows)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return [tuple(int(w, 16) for w in line.split()) for line in out.strip().splitlines()]

    return run


def test_philox_matches_rocrand(philox_ref):
    rng = np.random.default_rng(7)
    rows = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6]
    rows += [tuple(int(v) for v in rng.integers(0, 2**32, size=6, dtype=np.uint64)) for _ in range(200)]
    ref = philox_ref(rows)
    arr = np.array(rows, dtype=np.uint64)
    out = oracle.philox4x32_10(*[arr[:, i] for i in range(6)])
    got = list(zip(*[o.tolist() for o in out]))
    assert got == ref


def test_mask_words_match_rocrand(philox_ref):
    K, H, W, p, seed, draw, n = 5, 3, 7, 0.37, 0x123456789ABCDEF0, 9, 4
    S = oracle.bernoulli_mask(K, H, W, p, seed, draw, n)
    thr = sample_threshold(p)
    rows, coords = [], []
    for y in range(H):
        for x in range(W):
            for k in range(K):
                l = (y * W + x) * K + k
                q = l >> 2
                rows.append((q & 0xFFFFFFFF, q >> 32, n, draw, seed & 0xFFFFFFFF, seed >> 32))
                coords.append((k, y, x, l & 3))
    ref = philox_ref(rows)
    for (k, y, x, j), words in zip(coords, ref):
        assert S[k, y, x] == (words[j] < thr)


def test_threshold_exact():
    assert sample_threshold(1.0) == 2**32
    assert sample_threshold(0.5) == 2**31
    assert sample_threshold(0.1) == math.floor(0.1 * 2**32)
    with pytest.raises(ValueError):
        sample_threshold(0.0)
    with pytest.raises(ValueError):
        sample_threshold(1.5)


@pytest.mark.parametrize("p", [0.05, 0.1, 0.5, 0.9])
def test_mask_fraction_binomial(p):
    K, H, W = 8, 40, 50
    S = oracle.bernoulli_mask(K, H, W, p, seed=99, draw=1, image_index=0)
    n = S.size
    mean = n * p
    sd = math.sqrt(n * p * (1 - p))
    assert abs(S.sum() - mean) < 5 * sd


def test_mask_draws_independent():
    K, H, W, p = 8, 40, 50, 0.3
    a = oracle.bernoulli_mask(K, H, W, p, 5, 1, 0)
    b = oracle.bernoulli_mask(K, H, W, p, 5, 2, 0)
    c = oracle.bernoulli_mask(K, H, W, p, 5, 1, 1)
    n = a.size
    for other in (b, c):
        both = np.logical_and(a, other).sum()
        sd = math.sqrt(n * p * p * (1 - p * p))
        assert abs(both - n * p * p) < 5 * sd
    # same arguments give the same selection
    np.testing.assert_array_equal(a, oracle.bernoulli_mask(K, H, W, p, 5, 1, 0))


def test_mask_p1_selects_all():
    S = oracle.bernoulli_mask(3, 9, 11, 1.0, 1, 1, 0)
    assert S.all()
