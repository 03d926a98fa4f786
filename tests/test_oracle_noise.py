"""Pins for the oracle's Z(4) noise (CPU).

SplitMix64 reference outputs: the five first outputs for seed 1234567 as
published with Vigna's splitmix64.c test and reproduced in the Rosetta Code
task "Pseudo-random numbers/Splitmix64" (tests/golden/splitmix64.txt).
"""
import os

import numpy as np

from oracle import noise

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def _golden():
    vals = []
    seed = None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split("=")
        if k.strip() == "seed":
            seed = int(v)
        else:
            vals.append(int(v))
    return seed, vals


def test_splitmix64_published_outputs():
    seed, vals = _golden()
    out = noise.splitmix64(seed, np.arange(len(vals)))
    assert [int(v) for v in out] == vals


def test_z4_values_and_indexing():
    dims = (2, 2, 2, 4)
    eta = noise.z4_noise(7, dims, 3, 2)
    assert eta.shape == (2, 4, 2, 2, 2, 4, 3)
    assert np.allclose(np.abs(eta), 1.0)
    codes = noise.z4_codes(7, dims, 3, 2)
    # element (rhs 1, t=2, z=1, y=0, x=1, spin 3, colour 2) is counter (3+1)*Nvec + i
    nvec = 12 * 32
    s = 1 + 2 * (0 + 2 * (1 + 2 * 2))
    i = (s * 4 + 3) * 3 + 2
    ref = int(noise.splitmix64(7, np.array([4 * nvec + i]))[0]) >> 62
    assert codes[1, 2, 1, 0, 1, 3, 2] == ref
    # independent of how the stream is split into calls
    a = noise.z4_codes(7, dims, 3, 2)
    b = np.concatenate([noise.z4_codes(7, dims, 3, 1), noise.z4_codes(7, dims, 4, 1)])
    assert np.array_equal(a, b)


def test_z4_moments():
    """<eta> = 0, <eta^2> = 0, <|eta|^2> = 1 and uniform codes (Eqs. (3)-(4))."""
    dims = (4, 4, 4, 4)
    codes = noise.z4_codes(11, dims, 0, 64).ravel()
    n = codes.size
    counts = np.bincount(codes, minlength=4)
    chi2 = ((counts - n / 4) ** 2 / (n / 4)).sum()
    assert chi2 < 16.3  # 3 dof, p ~ 0.001
    eta = noise.z4_noise(11, dims, 0, 64).ravel()
    assert abs(eta.mean()) < 5 / np.sqrt(n)
    assert abs((eta ** 2).mean()) < 5 / np.sqrt(n)
    # <eta_i eta_j^*> = delta_ij: neighbouring components uncorrelated
    assert abs(np.mean(eta[1:] * np.conj(eta[:-1]))) < 5 / np.sqrt(n)
