"""Pins for the oracle's noise generator: Philox4x32-10 against rocRAND's
independent implementation, and the Gaussian draws against their defining
moments (<eta_a eta_b> = 2 delta_ab for the Langevin noise)."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _rocrand_ref(tmp_path, cases):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "philox_ref")
    subprocess.check_call([hipcc, "-O1", os.path.join(HERE, "philox_rocrand_ref.cpp"), "-o", exe])
    inp = "".join("%x %x %x %x %x %x\n" % tuple(c) for c in cases)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [[int(w, 16) for w in line.split()] for line in out.strip().splitlines()]


def test_philox_matches_rocrand(orc, tmp_path):
    rng = np.random.default_rng(7)
    # rocRAND takes the low counter pair as a 64-bit offset of 4*(c0 + 2^32 c1),
    # so c1 stays below 2^30 here
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF,
                                  0xFFFFFFFF), (1, 2, 3, 4, 5, 6)]
    for _ in range(60):
        c = [int(v) for v in rng.integers(0, 2**32, 6, dtype=np.uint64)]
        c[1] &= 0x3FFFFFFF
        cases.append(tuple(c))
    # the counters the library uses: (4*site + mu, step, draw, tag), key = seed
    for s, mu, n, j, tag in [(0, 0, 0, 0, 0), (1000, 3, 17, 3, 0), (77, 2, 0, 7, 1)]:
        cases.append((4 * s + mu, n, j, tag, 0xDEADBEEF, 0x12345678))
    ref = _rocrand_ref(tmp_path, cases)
    for c, r in zip(cases, ref):
        assert orc.philox4x32_10(c[:4], c[4:]) == r, c


def test_philox_counter_sensitivity(orc):
    base = orc.philox4x32_10([0, 0, 0, 0], [1, 0])
    for i in range(4):
        c = [0, 0, 0, 0]
        c[i] = 1
        assert orc.philox4x32_10(c, [1, 0]) != base
    assert orc.philox4x32_10([0, 0, 0, 0], [2, 0]) != base


def test_normal_pair_from_words(orc):
    """Box-Muller of the 53-bit uniforms built from the Philox words."""
    seed = 0x0123456789ABCDEF
    for c in [(0, 0, 0, 0), (5, 9, 2, 1), (123456, 7, 3, 0)]:
        w = orc.philox4x32_10(list(c), [seed & 0xFFFFFFFF, seed >> 32])
        uA = ((w[0] >> 5) * 2.0**26 + (w[1] >> 6) + 0.5) * 2.0**-53
        uB = ((w[2] >> 5) * 2.0**26 + (w[3] >> 6) + 0.5) * 2.0**-53
        assert 0.0 < uA < 1.0 and 0.0 < uB < 1.0
        r = np.sqrt(-2 * np.log(uA))
        n = orc.normal_pair(seed, *c)
        np.testing.assert_allclose(n, [r * np.cos(2 * np.pi * uB), r * np.sin(2 * np.pi * uB)],
                                   rtol=1e-14, atol=1e-15)


def test_langevin_noise_moments(orc):
    dims = (16, 16, 16, 8)  # 131072 links
    eta = orc.cl_noise_field(dims, 12345, 3).reshape(-1, 8)
    n = eta.shape[0]
    cov = eta.T @ eta / n
    se = np.sqrt(2 * 4.0 / n)  # std error of a variance estimate of N(0, 2)
    np.testing.assert_allclose(np.diag(cov), 2.0, atol=5 * se * 1.5)
    off = cov - np.diag(np.diag(cov))
    assert np.max(np.abs(off)) < 5 * np.sqrt(4.0 / n)
    assert np.max(np.abs(eta.mean(0))) < 5 * np.sqrt(2.0 / n)
    # Gaussian shape
    ks = scipy.stats.kstest(eta[:, 0] / np.sqrt(2), "norm")
    assert ks.pvalue > 1e-3
    # different steps and seeds give different noise
    assert not np.allclose(orc.cl_noise(12345, 0, 0, 3), orc.cl_noise(12345, 0, 0, 4))
    assert not np.allclose(orc.cl_noise(12345, 0, 0, 3), orc.cl_noise(12346, 0, 0, 3))
    np.testing.assert_array_equal(eta[5], orc.cl_noise(12345, 1, 1, 3))
