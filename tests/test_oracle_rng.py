"""Pins of the oracle's counter-based generator and normal transform.

* Philox4x32-10 words against rocRAND's independent implementation (its
  header-only engine compiled for the host and run on the CPU).
* Box-Muller: exact special cases of the 23-bit uniform mapping, and the
  distribution of 10^6 normals (moments, KS test against N(0,1)).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_rocrand")
    subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O1", "-o", exe,
                    os.path.join(HERE, "helpers", "philox_rocrand.cpp")], check=True, capture_output=True)

    def run(keys, ctrs):
        lines = "\n".join(" ".join(str(int(v)) for v in list(k) + list(c)) for k, c in zip(keys, ctrs))
        out = subprocess.run([exe], input=lines + "\n", capture_output=True, text=True, check=True).stdout
        return np.array([[int(v) for v in ln.split()] for ln in out.strip().splitlines()], dtype=np.uint64)
    return run


def test_philox_matches_rocrand(oracle_mod, rocrand_philox):
    rng = np.random.default_rng(0)
    n = 2000
    keys = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64)
    ctrs = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64)
    ctrs[:, 1] %= 2 ** 30                       # offset must fit 64 bits in the helper
    ctrs[:10] = 0                               # zero counter
    keys[:5] = 0
    ctrs[10:20, 0] = np.arange(10)              # the layout the solver uses: (k/2, path, node, tag)
    ctrs[10:20, 1:] = [7, 31, 0]
    ref = rocrand_philox(keys, ctrs)
    got = oracle_mod.philox(ctrs.astype(np.uint32), keys.astype(np.uint32)).astype(np.uint64)
    assert np.array_equal(got, ref)


def test_philox_word_uniformity(oracle_mod):
    n = 1 << 16
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n)
    out = oracle_mod.philox(ctr, np.zeros((n, 2), dtype=np.uint32))
    u = (out >> 8).astype(np.float64) / 2 ** 24
    ul = (out & 0x7FFFFF).astype(np.float64) / 2 ** 23     # the bits Box-Muller takes
    for c in range(4):
        assert stats.kstest(u[:, c], "uniform").pvalue > 1e-3
        assert stats.kstest(ul[:, c], "uniform").pvalue > 1e-3
    # bits are balanced
    bits = np.unpackbits(out.view(np.uint8)).mean()
    assert abs(bits - 0.5) < 1e-3


def test_box_muller_special_cases(oracle_mod):
    # the low 23 bits m of each word: ra with m = 0 -> u1 = 1 -> radius 0
    # (the high bits are ignored); m = 2^23 - 1 -> u1 = 2^-23 -> radius
    # sqrt(46 ln 2); rb with m = 0 -> angle 0, m = 2^21 (u2 = 1/4) -> pi/2,
    # m = 2^22 -> pi
    z = oracle_mod.normals([0xFF800000, 0x7FFFFF, 0xFFFFFFFF, 0x007FFFFF],
                           [123, 0xFF800000, 1 << 21, (1 << 22) | (1 << 31)])
    assert np.all(z[0] == 0.0)
    r = np.sqrt(46 * np.log(2.0))
    assert np.allclose(z[1], [r, 0.0], atol=1e-15)
    assert np.allclose(z[2], [0.0, r], atol=1e-14)
    assert np.allclose(z[3], [-r, 0.0], atol=1e-14)


def test_box_muller_distribution(oracle_mod):
    n = 1 << 19
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 3] = 5
    w = oracle_mod.philox(ctr, np.tile(np.array([[17, 29]], dtype=np.uint32), (n, 1)))
    z = np.concatenate([oracle_mod.normals(w[:, 0], w[:, 1]), oracle_mod.normals(w[:, 2], w[:, 3])]).ravel()
    m = z.size
    assert abs(z.mean()) < 5 / np.sqrt(m)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / m)
    assert abs(stats.skew(z)) < 5 * np.sqrt(6 / m)
    assert abs(stats.kurtosis(z)) < 5 * np.sqrt(24 / m)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # the two normals of a pair are uncorrelated
    zz = oracle_mod.normals(w[:, 0], w[:, 1])
    assert abs(np.corrcoef(zz[:, 0], zz[:, 1])[0, 1]) < 5 / np.sqrt(n)
