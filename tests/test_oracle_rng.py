"""Pins for the oracle's noise: Philox4x32-10 words and Box-Muller normals.

Philox is pinned bit-for-bit to rocRAND's engine (an independent
implementation of the same published generator, compiled here from its
header and run on the host).  The normals are pinned to N(0,1) by a
Kolmogorov-Smirnov test and by moment and independence checks, and the
per-step draw used by the stepping code is tied to the single-face
definition through a one-step run.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats as sps

import oracle

PIN_SRC = os.path.join(os.path.dirname(__file__), "pins", "rocrand_philox.cpp")


@pytest.fixture(scope="module")
def rocrand_exe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    d = tempfile.mkdtemp(prefix="she_pin_")
    exe = os.path.join(d, "rocrand_philox")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", PIN_SRC, "-o", exe],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_exe):
    rng = np.random.default_rng(12345)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (1, 0, 0, 0, 0, 0), (0, 0, 1, 0, 0, 0),
             (0, 0, 0, 1, 0, 0), (0, 0, 0, 0, 1, 0), (0, 0, 0, 0, 0, 1),
             (0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344, 0xA4093822, 0x299F31D0)]
    for _ in range(300):
        cases.append(tuple(int(v) for v in rng.integers(0, 2 ** 32, size=6, dtype=np.uint64)))
    inp = "".join("%d %d %d %d %d %d\n" % c for c in cases)
    out = subprocess.run([rocrand_exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [tuple(int(v) for v in line.split()) for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for (k0, k1, c0, c1, c2, c3), want in zip(cases, ref):
        got = tuple(int(v) for v in oracle.philox([c0, c1, c2, c3], [k0, k1]))
        assert got == want, (k0, k1, c0, c1, c2, c3)


def test_philox_is_not_identity_and_avalanches():
    a = oracle.philox([0, 0, 0, 0], [0, 0])
    b = oracle.philox([1, 0, 0, 0], [0, 0])
    flips = sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b))
    assert 40 < flips < 88  # ~64 of 128 bits change for a one-bit counter change


def test_normals_distribution():
    z = np.concatenate([oracle.normals(7, rz, 0, step, 0, 20000) for rz in range(3) for step in (0, 1, 2 ** 33 + 5)])
    n = z.size
    ks = sps.kstest(z, "norm")
    assert ks.pvalue > 1e-4, ks
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(sps.skew(z)) < 5 * np.sqrt(6.0 / n)
    assert abs(sps.kurtosis(z)) < 5 * np.sqrt(24.0 / n)
    # the two members of a Box-Muller pair and neighbouring pairs are uncorrelated
    q = z[: (n // 4) * 4].reshape(-1, 4)
    for a, b in ((0, 1), (2, 3), (1, 2), (0, 2)):
        c = np.corrcoef(q[:, a], q[:, b])[0, 1]
        assert abs(c) < 5 / np.sqrt(q.shape[0])
    # every lane on its own is standard normal
    for lane in range(4):
        assert sps.kstest(q[:, lane], "norm").pvalue > 1e-4


def test_streams_are_distinct():
    base = oracle.normals(0, 0, 0, 0, 0, 4096)
    for other in (oracle.normals(1, 0, 0, 0, 0, 4096), oracle.normals(0, 1, 0, 0, 0, 4096),
                  oracle.normals(0, 0, 1, 0, 0, 4096), oracle.normals(0, 0, 0, 1, 0, 4096),
                  oracle.normals(0, 0, 0, 2 ** 32, 0, 4096)):
        assert abs(np.corrcoef(base, other)[0, 1]) < 0.08
        assert not np.any(base == other)


def test_step_uses_face_definition():
    """One FE step with r = 0 on a uniform periodic rod changes cell i by
    sigma*u0*(z_{i+1} - z_i); the z's must be the single-face definition."""
    N, sigma, u0, n = 12, 0.3, 2.0, 5
    d = oracle.Desc(dim=1, n=(N, 1, 1), r=0.0, sigma=sigma, u0=u0, seed=3, realisation=9)
    u = oracle.init(d)
    oracle.advance(d, u, n, 1)
    z = oracle.normals(3, 9, 0, n, 0, N)
    want = u0 + sigma * u0 * (np.roll(z, -1) - z)
    np.testing.assert_allclose(u, want, rtol=0, atol=1e-15)


def test_init_perturbation_uses_tag1():
    d = oracle.Desc(dim=2, n=(8, 4, 1), r=0.1, sigma=0.1, u0=1.0, init_sd=0.25, seed=11, realisation=4)
    u = oracle.init(d)
    z = oracle.normals(11, 4, 1, 0, 0, 32)
    np.testing.assert_allclose(u, 1.0 + 0.25 * z, rtol=0, atol=1e-15)
