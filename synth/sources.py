"""Even-site source vectors phi of shape (n, Vh, 4, 3), complex128.

The solver's right-hand side is b = A^dag phi; that product is the solver's own
arithmetic and is formed by its caller, not here.
"""
import numpy as np


def _vh(dims):
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    return Lx * Ly * Lz * Lt // 2


def point_sources(dims, n=12):
    """Point sources at the origin (an even site, even index 0).

    Source j has a 1 at (spin, colour) = divmod(j, 3): j = 0 is (Dirac, colour) = (1, 1)
    of the paper's first source and j = 1 its second, (1, 2).
    """
    if not 1 <= n <= 12:
        raise ValueError("point sources: 1 <= n <= 12")
    phi = np.zeros((n, _vh(dims), 4, 3), dtype=np.complex128)
    for j in range(n):
        s, c = divmod(j, 3)
        phi[j, 0, s, c] = 1.0
    return phi


def gaussian_sources(dims, n, rng):
    """i.i.d. complex normal components with E|phi|^2 = 1: (N(0,1) + i N(0,1))/sqrt(2)."""
    shape = (n, _vh(dims), 4, 3)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def z2_sources(dims, n, rng):
    """Real Z2 noise: each of the 12 components of every even site is +1 or -1 with probability 1/2."""
    shape = (n, _vh(dims), 4, 3)
    bits = rng.integers(0, 2, size=shape)
    return (1.0 - 2.0 * bits).astype(np.complex128)
