"""Pins of the oracle's seeding of the indefinite system gamma5 A x = gamma5 phi (oracle/seedminres.py), CPU only.

Independent references: a Krylov basis of H built by numpy's QR from the powers H^k r_0 (no
Lanczos), and numpy's least-squares and dense solves.
  * H is Hermitian and indefinite on this system (eigenvalues of both signs);
  * the RHS-1 iterate after i steps minimises ||c - H x|| over x_0 + K_i(H, r_0) (the defining
    property of MINRES), and its residual estimate equals the true residual;
  * the seeded iterate of RHS j minimises the part of its residual inside K_{i+1}(H, r_0^1);
  * a duplicate of RHS 1 is seeded to the RHS-1 iterate;
  * the finished solutions solve A x = phi to tol and agree with the dense solve to 1e-8, and
    reach the same x as the normal system M x = A^dag phi.
A dropped eps or delta term, a wrong rotation sign or a conjugation missing in eta breaks one of them.
"""
import numpy as np
import pytest

from oracle import seedminres as smr
from oracle.wilson import WilsonEO, dense, flat, matvec_H, matvec_M
from synth.links import random_su3_links

DIMS = (4, 2, 2, 4)


@pytest.fixture(scope="module")
def system():
    U = random_su3_links(DIMS, 0.5, np.random.default_rng(71))
    op = WilsonEO(U, DIMS, 0.18)
    H = matvec_H(op)
    N = 12 * op.Vh
    Hd = dense(H, N)
    rng = np.random.default_rng(72)
    phi = rng.standard_normal((3, op.Vh, 4, 3)) + 1j * rng.standard_normal((3, op.Vh, 4, 3))
    C = flat(phi * np.array([1, 1, -1, -1])[:, None])      # gamma5 phi
    return dict(op=op, H=H, Hd=Hd, N=N, C=C, phi=flat(phi))


def _krylov(Hd, r0, n):
    """Orthonormal basis (columns) of K_n(H, r0) from the powers of H, by numpy's QR."""
    K = np.empty((r0.size, n), dtype=np.complex128)
    K[:, 0] = r0 / np.linalg.norm(r0)
    for j in range(1, n):
        y = Hd @ K[:, j - 1]
        K[:, j] = y / np.linalg.norm(y)
    Q, _ = np.linalg.qr(K)
    return Q


def test_h_is_hermitian_and_indefinite(system):
    Hd = system["Hd"]
    assert np.max(np.abs(Hd - Hd.conj().T)) <= 1e-13 * np.max(np.abs(Hd))
    lam = np.linalg.eigvalsh(0.5 * (Hd + Hd.conj().T))
    assert lam[0] < 0 < lam[-1]


@pytest.mark.parametrize("steps", [1, 2, 3, 5, 8])
def test_rhs1_iterate_minimises_the_residual(system, steps):
    Hd, C = system["Hd"], system["C"]
    out = smr.seed_minres(system["H"], C, k=1, tol=1e-300, past=0.0, m=steps)
    assert out["m"] == steps
    Q = _krylov(Hd, C[0], steps)
    y, *_ = np.linalg.lstsq(Hd @ Q, C[0], rcond=None)
    x_ref = Q @ y
    assert np.linalg.norm(out["X"][0] - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    true = np.linalg.norm(C[0] - Hd @ out["X"][0]) / np.linalg.norm(C[0])
    assert abs(out["est"][-1] - true) <= 1e-9 * max(true, 1e-12)


@pytest.mark.parametrize("steps", [2, 4, 7])
def test_seeded_iterate_is_the_projected_minimal_residual(system, steps):
    Hd, C = system["Hd"], system["C"]
    out = smr.seed_minres(system["H"], C, k=1, tol=1e-300, past=0.0, m=steps)
    Q1 = _krylov(Hd, C[0], steps + 1)
    Q = Q1[:, :steps]
    for j in (1, 2):
        y, *_ = np.linalg.lstsq(Q1.conj().T @ Hd @ Q, Q1.conj().T @ C[j], rcond=None)
        x_ref = Q @ y
        assert np.linalg.norm(out["X"][j] - x_ref) <= 1e-9 * np.linalg.norm(x_ref), j


def test_duplicate_rhs_is_seeded_to_the_rhs1_iterate(system):
    C = system["C"]
    D = np.stack([C[0], C[0], C[1]])
    out = smr.seed_minres(system["H"], D, k=5, tol=1e-10, past=1.5)
    assert np.linalg.norm(out["X"][1] - out["X"][0]) <= 1e-12 * np.linalg.norm(out["X"][0])


def test_solutions_match_the_dense_and_the_normal_system(system):
    op, Hd, C = system["op"], system["Hd"], system["C"]
    out = smr.solve_indefinite(system["H"], C, k=10, tol=1e-10)
    assert np.all(out["relres"] <= 1e-10), out["relres"]
    xs = np.linalg.solve(Hd, C.T).T
    err = np.linalg.norm(out["X"] - xs, axis=1) / np.linalg.norm(xs, axis=1)
    assert np.all(err <= 1e-8), err
    # the same x solves the normal system M x = A^dag phi (gamma5 A^dag ... = H^dag H)
    M = matvec_M(op)
    b = flat(op.apply_Adag(system["phi"].reshape(3, op.Vh, 4, 3)))
    res = np.linalg.norm(b - M(out["X"]), axis=1) / np.linalg.norm(b, axis=1)
    assert np.all(res <= 1e-8), res
    # seeding helped: the later systems need fewer MINRES iterations than RHS 1 needed Lanczos steps
    assert max(out["iters"][1:]) < out["m"]


def test_qr_seeding_pays_with_isolated_low_modes():
    """As for Seed-CG: on 4^4 with the flux background at kappa 0.16 (six near-zero modes apart from
    the bulk) the minimal-residual seeding halves MINRES (seeded at most 0.6x a cold start: 72
    against 140); on the same links without the flux it saves little (at least 0.85x: 88-90
    against 100-102)."""
    from dataclasses import replace

    from oracle.wilson import WilsonEO, flat, gamma5, matvec_H
    from synth.configs import CONFIGS, make_links, make_sources
    for flux, lo, hi in (((1, 1), 0.0, 0.6), (None, 0.85, 1.0)):
        cfg = replace(CONFIGS["c1"], flux=flux)
        op = WilsonEO(make_links(cfg), cfg.dims, 0.16)
        H = matvec_H(op)
        C = flat(gamma5(make_sources(cfg)))
        ref = smr.seed_minres(H, C, k=10, tol=1e-10, past=1.5)
        for j in range(1, C.shape[0]):
            _, it_s, r_s = smr.minres(H, C[j], ref["X"][j], tol=1e-10)
            _, it_c, r_c = smr.minres(H, C[j], None, tol=1e-10)
            assert r_s <= 1e-10 and r_c <= 1e-10
            assert lo <= it_s / it_c <= hi, (flux, j, it_s, it_c)
