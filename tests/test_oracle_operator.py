"""Pins of the oracle's Wilson operator against the mathematics (CPU only).

Each test checks something the definition of section 3 of the paper fixes:
the Clifford algebra, the closed-form free-field spectra, gamma5-hermiticity,
Hermiticity/positivity of M, gauge covariance, and a second dense construction.
"""
import numpy as np
import pytest

from oracle import dense as dn
from oracle.wilson import WilsonEO, dense, flat, gamma5
from synth.links import random_su3_links


def _full_dense_from_stencil(op, dims):
    ie, io = dn.parity_split(dims)

    def applyD(X):
        n = X.shape[0]
        xe = X[:, ie].reshape(n, op.Vh, 4, 3)
        xo = X[:, io].reshape(n, op.Vh, 4, 3)
        ye, yo = op.apply_D(xe, xo)
        Y = np.zeros_like(X)
        Y[:, ie] = ye.reshape(n, -1)
        Y[:, io] = yo.reshape(n, -1)
        return Y

    return dense(applyD, 12 * op.V)


def _eo_dense(op, which):
    fn = {"A": op.apply_A, "Adag": op.apply_Adag, "M": op.apply_M}[which]
    n = 12 * op.Vh
    return dense(lambda X: flat(fn(X.reshape(-1, op.Vh, 4, 3))), n)


def test_gamma_clifford_and_gamma5():
    g = dn.gamma_matrices()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2.0 * (mu == nu) * np.eye(4), atol=1e-15)
    assert np.allclose(dn.gamma5(), np.diag([1, 1, -1, -1]), atol=1e-15)


@pytest.mark.parametrize("dims,t_bc", [((2, 2, 2, 2), -1), ((4, 2, 2, 4), -1), ((2, 4, 2, 2), 1),
                                       ((4, 4, 2, 2), -1)])
def test_stencil_matches_dense_formula(dims, t_bc):
    rng = np.random.default_rng(11)
    U = random_su3_links(dims, 0.7, rng)
    op = WilsonEO(U, dims, 0.137, t_bc=t_bc)
    D1 = _full_dense_from_stencil(op, dims)
    D2 = dn.dense_D(U, dims, 0.137, t_bc=t_bc)
    assert np.max(np.abs(D1 - D2)) < 1e-15


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4)])
@pytest.mark.parametrize("kappa", [0.09, 0.124])
def test_free_field_full_spectrum(dims, kappa):
    V = int(np.prod(dims))
    U = np.tile(np.eye(3, dtype=np.complex128), (4, V, 1, 1))
    op = WilsonEO(U, dims, kappa)
    D = _full_dense_from_stencil(op, dims)
    lam = np.sort(np.linalg.eigvalsh(D.conj().T @ D))
    ref = dn.free_spectrum_DdagD(dims, kappa)
    assert np.max(np.abs(lam - ref) / ref) < 1e-12


@pytest.mark.parametrize("dims,t_bc", [((2, 2, 2, 2), -1), ((4, 4, 2, 4), -1), ((4, 4, 4, 4), -1),
                                       ((4, 2, 2, 2), 1)])
def test_free_field_eo_spectrum(dims, t_bc):
    V = int(np.prod(dims))
    kappa = 0.11
    U = np.tile(np.eye(3, dtype=np.complex128), (4, V, 1, 1))
    op = WilsonEO(U, dims, kappa, t_bc=t_bc)
    M = _eo_dense(op, "M")
    lam = np.sort(np.linalg.eigvalsh(0.5 * (M + M.conj().T)))
    ref = dn.free_spectrum_eo(dims, kappa, t_bc=t_bc)
    assert lam.shape == ref.shape
    assert np.max(np.abs(lam - ref) / ref) < 1e-11


def test_gamma5_hermiticity_and_M_hpd():
    dims = (4, 2, 2, 4)
    rng = np.random.default_rng(5)
    U = random_su3_links(dims, 0.9, rng)
    op = WilsonEO(U, dims, 0.15)
    D = _full_dense_from_stencil(op, dims)
    G5 = np.kron(np.eye(op.V), np.kron(np.diag([1.0, 1, -1, -1]), np.eye(3)))
    assert np.max(np.abs(D.conj().T - G5 @ D @ G5)) < 1e-15
    A = _eo_dense(op, "A")
    Ad = _eo_dense(op, "Adag")
    assert np.max(np.abs(Ad - A.conj().T)) < 1e-14
    M = _eo_dense(op, "M")
    assert np.max(np.abs(M - M.conj().T)) < 1e-14 * np.max(np.abs(M))
    assert np.max(np.abs(M - A.conj().T @ A)) < 1e-13
    lam = np.linalg.eigvalsh(0.5 * (M + M.conj().T))
    assert lam.min() > 0


def test_schur_complement_and_eo_solve():
    dims = (4, 2, 2, 4)
    rng = np.random.default_rng(6)
    U = random_su3_links(dims, 0.5, rng)
    kappa = 0.13
    op = WilsonEO(U, dims, kappa)
    D = dn.dense_D(U, dims, kappa)
    A_dense = dn.dense_A(D, dims)
    A = _eo_dense(op, "A")
    assert np.max(np.abs(A - A_dense)) < 1e-14
    # full solve D x = eta equals the even-odd solve A x_e = phi_e, x_o = eta_o + kappa H_oe x_e
    eta = rng.standard_normal(12 * op.V) + 1j * rng.standard_normal(12 * op.V)
    x_full = np.linalg.solve(D, eta)
    ie, io = dn.parity_split(dims)
    eta_e = eta[ie].reshape(op.Vh, 4, 3)
    eta_o = eta[io].reshape(op.Vh, 4, 3)
    phi = op.eo_source(eta_e, eta_o)
    x_e = np.linalg.solve(A, phi.ravel()).reshape(op.Vh, 4, 3)
    x_o = op.reconstruct_odd(x_e, eta_o)
    assert np.max(np.abs(x_e.ravel() - x_full[ie])) < 1e-12
    assert np.max(np.abs(x_o.ravel() - x_full[io])) < 1e-12


def test_gauge_covariance():
    """D[U^Omega] (Omega psi) = Omega D[U] psi with U^Omega_mu(n) = Omega(n) U_mu(n) Omega(n+mu)^dag."""
    dims = (4, 4, 2, 4)
    V = int(np.prod(dims))
    rng = np.random.default_rng(7)
    U = random_su3_links(dims, 0.8, rng)
    Om = random_su3_links(dims, 2.0, rng)[0]            # (V, 3, 3) random SU(3)
    C = dn.coords(dims)
    Ug = np.empty_like(U)
    for mu in range(4):
        nb = C.copy()
        nb[:, mu] = (nb[:, mu] + 1) % dims[mu]
        fwd = dn.site_index(nb, dims)
        Ug[mu] = Om @ U[mu] @ np.conj(np.swapaxes(Om[fwd], -1, -2))
    kappa = 0.14
    op = WilsonEO(U, dims, kappa)
    opg = WilsonEO(Ug, dims, kappa)
    ie_sites = np.nonzero(C.sum(1) % 2 == 0)[0]
    Om_e = Om[ie_sites]
    psi = rng.standard_normal((op.Vh, 4, 3)) + 1j * rng.standard_normal((op.Vh, 4, 3))
    rot = lambda x: np.einsum("sab,sib->sia", Om_e, x)
    lhs = opg.apply_M(rot(psi))
    rhs = rot(op.apply_M(psi))
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * np.max(np.abs(rhs))


def test_gamma5_in_oracle_is_diag():
    x = np.ones((3, 4, 3), dtype=np.complex128)
    y = gamma5(x)
    assert np.all(y[:, :2] == 1) and np.all(y[:, 2:] == -1)
