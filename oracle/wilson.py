"""Even-odd Wilson operators of section 3 of the paper, on top of the plain C hop.

  H_eo, H_oe : parity blocks of the hopping term H (wilson_ref.c)
  A    = 1 - kappa^2 H_eo H_oe       (Schur complement on the even sites)
  A^dag = gamma5 A gamma5
  M    = A^dag A                      (the Hermitian positive-definite normal system)
  D    = [[1, -kappa H_eo], [-kappa H_oe, 1]] on (even, odd) for full-lattice checks

Vectors are complex128 arrays (..., Vh, 4, 3); leading axes are batches of vectors.
"""
import ctypes

import numpy as np

from . import _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build()
        lib = ctypes.CDLL(path)
        lib.oracle_hop.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64]
        lib.oracle_hop.restype = None
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads():
    return int(_load().oracle_num_threads())


GAMMA5_DIAG = np.array([1.0, 1.0, -1.0, -1.0])


def gamma5(x):
    """gamma5 = diag(1, 1, -1, -1) on the spin index."""
    return x * GAMMA5_DIAG[:, None]


class WilsonEO:
    def __init__(self, links, dims, kappa, t_bc=-1):
        self.dims = tuple(int(d) for d in dims)
        if any(d % 2 for d in self.dims) or any(d < 2 for d in self.dims):
            raise ValueError("every lattice extent must be even and >= 2")
        self.V = int(np.prod(self.dims))
        self.Vh = self.V // 2
        self.kappa = float(kappa)
        self.t_bc = int(t_bc)
        self.U = np.ascontiguousarray(links, dtype=np.complex128).reshape(4, self.V, 3, 3)
        self._dims_c = (ctypes.c_int32 * 4)(*self.dims)

    def hop(self, x, out_parity):
        """H_{p,1-p} x: x lives on parity 1-p, the result on parity p."""
        x = np.ascontiguousarray(x, dtype=np.complex128)
        lead = x.shape[:-3]
        assert x.shape[-3:] == (self.Vh, 4, 3), x.shape
        nvec = int(np.prod(lead)) if lead else 1
        out = np.empty_like(x)
        _load().oracle_hop(self._dims_c, self.t_bc, self.U.ctypes.data, x.ctypes.data,
                           out.ctypes.data, int(out_parity), nvec)
        return out

    def H_eo(self, x_odd):
        return self.hop(x_odd, 0)

    def H_oe(self, x_even):
        return self.hop(x_even, 1)

    def apply_A(self, x):
        return x - self.kappa ** 2 * self.H_eo(self.H_oe(x))

    def apply_Adag(self, x):
        return gamma5(self.apply_A(gamma5(x)))

    def apply_M(self, x):
        return self.apply_Adag(self.apply_A(x))

    def apply_D(self, x_even, x_odd):
        """Full Wilson D on (even, odd) halves."""
        return (x_even - self.kappa * self.H_eo(x_odd),
                x_odd - self.kappa * self.H_oe(x_even))

    def eo_source(self, eta_even, eta_odd):
        """phi_e = eta_e + kappa H_eo eta_o: the even-site source of the Schur system A x_e = phi_e."""
        return eta_even + self.kappa * self.H_eo(eta_odd)

    def reconstruct_odd(self, x_even, eta_odd):
        """x_o = eta_o + kappa H_oe x_e."""
        return eta_odd + self.kappa * self.H_oe(x_even)


def flat(x):
    """(..., Vh, 4, 3) -> (..., 12 Vh) view used by the solvers."""
    return x.reshape(x.shape[:-3] + (-1,))


def unflat(x, Vh):
    return x.reshape(x.shape[:-1] + (Vh, 4, 3))


def matvec_M(op):
    """M as a function on flattened vectors (one or a batch)."""
    def f(x):
        return flat(op.apply_M(unflat(x, op.Vh)))
    return f


def matvec_H(op):
    """H = gamma5 A (Hermitian, indefinite) as a function on flattened vectors (one or a batch)."""
    def f(x):
        return flat(gamma5(op.apply_A(unflat(x, op.Vh))))
    return f


def dense(fn, n):
    """Dense matrix of a linear map on C^n, built column by column from unit vectors."""
    cols = np.empty((n, n), dtype=np.complex128)
    eye = np.eye(n, dtype=np.complex128)
    for lo in range(0, n, 256):
        hi = min(lo + 256, n)
        cols[:, lo:hi] = fn(eye[lo:hi]).T
    return cols
