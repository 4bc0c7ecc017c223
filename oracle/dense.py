"""Dense Wilson-Dirac matrices written out from the definition (tiny lattices only).

This is a second, independent construction of the operator: it assembles the full
12V x 12V matrix block by block with Kronecker products of the NumPy gamma matrices
and the links, with its own site indexing.  The tests compare it with the C stencil
applied to unit vectors, and pin it against the closed-form free-field spectra.
"""
import numpy as np

# Pauli matrices and the Euclidean chiral gamma basis (Hermitian):
#   gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] for k = 1, 2, 3;  gamma_4 = [[0, 1], [1, 0]].
SIGMA = np.array([[[0, 1], [1, 0]],
                  [[0, -1j], [1j, 0]],
                  [[1, 0], [0, -1]]], dtype=np.complex128)


def gamma_matrices():
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    Z = np.zeros((2, 2))
    for k in range(3):
        g[k] = np.block([[Z, -1j * SIGMA[k]], [1j * SIGMA[k], Z]])
    g[3] = np.block([[Z, np.eye(2)], [np.eye(2), Z]])
    return g


def gamma5():
    g = gamma_matrices()
    return g[0] @ g[1] @ g[2] @ g[3]


def coords(dims):
    """Lexicographic coordinates: s = x + Lx (y + Ly (z + Lz t))."""
    Lx, Ly, Lz, Lt = dims
    s = np.arange(Lx * Ly * Lz * Lt)
    return np.stack([s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)], axis=1)


def site_index(c, dims):
    Lx, Ly, Lz, Lt = dims
    return c[..., 0] + Lx * (c[..., 1] + Ly * (c[..., 2] + Lz * c[..., 3]))


def dense_D(U, dims, kappa, t_bc=-1):
    """D = 1 - kappa sum_mu [(1-g_mu) (x) U_mu(n) delta_{n+mu,m} + (1+g_mu) (x) U_mu(m)^dag delta_{n-mu,m}]."""
    dims = tuple(int(d) for d in dims)
    V = int(np.prod(dims))
    U = np.asarray(U).reshape(4, V, 3, 3)
    g = gamma_matrices()
    I4 = np.eye(4)
    C = coords(dims)
    D = np.eye(12 * V, dtype=np.complex128)
    for n in range(V):
        for mu in range(4):
            fwd = C[n].copy()
            fwd[mu] = (fwd[mu] + 1) % dims[mu]
            bwd = C[n].copy()
            bwd[mu] = (bwd[mu] - 1) % dims[mu]
            sf = 1.0 if not (mu == 3 and C[n, 3] == dims[3] - 1) else float(t_bc)
            sb = 1.0 if not (mu == 3 and C[n, 3] == 0) else float(t_bc)
            m_f = site_index(fwd, dims)
            m_b = site_index(bwd, dims)
            D[12 * n:12 * n + 12, 12 * m_f:12 * m_f + 12] -= kappa * sf * np.kron(I4 - g[mu], U[mu, n])
            D[12 * n:12 * n + 12, 12 * m_b:12 * m_b + 12] -= kappa * sb * np.kron(
                I4 + g[mu], U[mu, m_b].conj().T)
    return D


def parity_split(dims):
    """Indices (into 12V) of the even and odd components, each in increasing site order."""
    C = coords(dims)
    par = C.sum(axis=1) % 2
    ev = np.nonzero(par == 0)[0]
    od = np.nonzero(par == 1)[0]
    comp = np.arange(12)
    return (ev[:, None] * 12 + comp).ravel(), (od[:, None] * 12 + comp).ravel()


def dense_eo_blocks(D, dims):
    """Return (D_ee, D_eo, D_oe, D_oo) of a full dense matrix."""
    ie, io = parity_split(dims)
    return D[np.ix_(ie, ie)], D[np.ix_(ie, io)], D[np.ix_(io, ie)], D[np.ix_(io, io)]


def dense_A(D, dims):
    """Schur complement A = D_ee - D_eo D_oo^{-1} D_oe (D_ee = D_oo = 1 for Wilson)."""
    Dee, Deo, Doe, Doo = dense_eo_blocks(D, dims)
    return Dee - Deo @ np.linalg.solve(Doo, Doe)


def free_spectrum_DdagD(dims, kappa, t_bc=-1):
    """Closed form of the free (U = 1) full D^dag D: (1 - 2k sum cos p)^2 + 4k^2 sum sin^2 p, 12-fold."""
    ps = _momenta(dims, t_bc)
    C = np.cos(ps).sum(axis=1)
    S2 = (np.sin(ps) ** 2).sum(axis=1)
    lam = (1.0 - 2.0 * kappa * C) ** 2 + 4.0 * kappa ** 2 * S2
    return np.sort(np.repeat(lam, 12))


def free_spectrum_eo(dims, kappa, t_bc=-1):
    """Closed form of the free even-odd A^dag A: |1 - 4 k^2 (C +/- i S)^2|^2, each sign 3-fold per momentum.

    C = sum_mu cos p_mu, S = (sum_mu sin^2 p_mu)^(1/2); every momentum p of the full
    lattice is listed, which counts each even-sublattice mode once per sign.
    """
    ps = _momenta(dims, t_bc)
    C = np.cos(ps).sum(axis=1)
    S = np.sqrt((np.sin(ps) ** 2).sum(axis=1))
    lam_p = np.abs(1.0 - 4.0 * kappa ** 2 * (C + 1j * S) ** 2) ** 2
    lam_m = np.abs(1.0 - 4.0 * kappa ** 2 * (C - 1j * S) ** 2) ** 2
    return np.sort(np.concatenate([np.repeat(lam_p, 3), np.repeat(lam_m, 3)]))


def _momenta(dims, t_bc):
    axes = []
    for mu, L in enumerate(dims):
        n = np.arange(L)
        if mu == 3 and t_bc == -1:
            axes.append((2 * n + 1) * np.pi / L)
        else:
            axes.append(2 * n * np.pi / L)
    grid = np.meshgrid(*axes, indexing="ij")
    return np.stack([a.ravel() for a in grid], axis=1)
