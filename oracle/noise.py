"""Z(4) noise (oracle; test infrastructure only).

Sec. 2 uses Z(N) noise with N = 4: every component is one of the fourth
roots of unity, independent, so <eta_i eta_j^*> = delta_ij and <eta> = 0
(Eqs. (3)-(4)).  The paper does not say how the noise is drawn; this project
fixes a counter-based generator so that any noise vector can be regenerated
anywhere, in any order, bit for bit:

  code(seed, n, i) = top two bits of the (n * Nvec + i)-th output of
                     SplitMix64 seeded with `seed`
  eta^(n)_i       = i^code         (values 1, i, -1, -i)

where Nvec = 12 V and i is the lexicographic vector index
(s * 4 + spin) * 3 + colour.  SplitMix64 is the generator of Steele, Lea and
Flood (OOPSLA 2014) in Vigna's public-domain formulation: the state advances
by the golden-ratio increment 0x9E3779B97F4A7C15 and each output is the
state passed through the 64-bit finaliser (xor-shift 30, multiply
0xBF58476D1CE4E5B9, xor-shift 27, multiply 0x94D049BB133111EB, xor-shift 31).
The c-th output (c = 0, 1, ...) therefore finalises seed + (c + 1) * gamma
modulo 2^64.

Pinned by tests/test_oracle_noise.py against published SplitMix64 outputs
and the Z(4) moments.
"""
import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, counters):
    """Outputs number `counters` (uint64 array) of SplitMix64 seeded with seed."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (c + np.uint64(1)) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * MIX1
        z = (z ^ (z >> np.uint64(27))) * MIX2
        z = z ^ (z >> np.uint64(31))
    return z


def z4_codes(seed, dims, first, nrhs):
    """Integer codes k in {0,1,2,3}, shape (nrhs, Lt, Lz, Ly, Lx, 4, 3), uint8."""
    Lx, Ly, Lz, Lt = dims
    nvec = 12 * Lx * Ly * Lz * Lt
    out = np.empty((nrhs, nvec), dtype=np.uint8)
    idx = np.arange(nvec, dtype=np.uint64)
    for r in range(nrhs):
        n = np.uint64(first + r)
        out[r] = (splitmix64(seed, n * np.uint64(nvec) + idx) >> np.uint64(62)).astype(np.uint8)
    return out.reshape((nrhs, Lt, Lz, Ly, Lx, 4, 3))


_ROOTS = np.array([1.0, 1.0j, -1.0, -1.0j], dtype=np.complex128)


def z4_noise(seed, dims, first, nrhs):
    """Noise vectors eta^(first..first+nrhs-1), complex128, lexicographic."""
    return _ROOTS[z4_codes(seed, dims, first, nrhs)]
