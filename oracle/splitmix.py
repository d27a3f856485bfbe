"""Counter-based random initial subspace (oracle side).

Test infrastructure only (see the package docstring).

The guide starts FEAST from a random subspace when no initial guess is given
(fpm(5)=0, Table tab_fpm; "Initial Guess | Random" in the HelloWorld output) but
does not say which distribution or generator.  Reading: entry t of the block is
drawn from SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): state_t = seed + (t + 1) * 0x9E3779B97F4A7C15 (mod 2^64),
mixed by the published finaliser, and mapped to [-1, 1) as 2 * (z >> 11) * 2^-53 - 1.
For a real n x m0 block, t = i + j * n (column-major).  For a complex block the
real part of entry (i, j) uses t = 2 (i + j n) and the imaginary part t = 2 (i + j n) + 1.
The HIP library implements the same published generator independently.

Probe block of the stochastic eigenvalue count (fpm(14)=2): real Rademacher entries,
+1 or -1 by the top bit of the same raw outputs (set -> -1), with t = i + j * n.
"""

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_raw(seed, count):
    """The first ``count`` 64-bit outputs of SplitMix64 started from ``seed``."""
    with np.errstate(over="ignore"):
        t = np.arange(1, count + 1, dtype=np.uint64)
        s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + t * _GAMMA
        z = s
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_uniform(seed, count):
    """Values 2*u - 1, u = (z >> 11) * 2^-53, for counters t = 0..count-1."""
    z = splitmix64_raw(seed, count)
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


def initial_subspace(n, m0, seed, is_complex):
    """The n x m0 random starting block (column-major counter order, see above)."""
    if is_complex:
        v = splitmix64_uniform(seed, 2 * n * m0)
        re = v[0::2].reshape(m0, n).T
        im = v[1::2].reshape(m0, n).T
        return (re + 1j * im).astype(np.complex128)
    v = splitmix64_uniform(seed, n * m0)
    return v.reshape(m0, n).T.astype(np.float64).copy()


def rademacher_block(n, m0, seed):
    """n x m0 block of +-1: -1 where the top bit of SplitMix64 output t = i + j n is set."""
    z = splitmix64_raw(seed, n * m0)
    v = np.where((z >> np.uint64(63)) != np.uint64(0), -1.0, 1.0)
    return v.reshape(m0, n).T.astype(np.float64).copy()
