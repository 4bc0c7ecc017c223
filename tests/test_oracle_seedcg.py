"""Pins of the oracle's Algorithm 1 (Seed-CG) and CG against the mathematics (CPU only).

  * Eq. (2): T = L U with the gamma/delta recurrences of its LU.
  * T from the CG coefficients (the Lanczos-CG correspondence, Saad 6.7.3).
  * The D-Lanczos iterate x^1 equals the CG iterate, and beta_i |zeta_i/delta_i| equals
    the true residual norm.
  * Eq. (1): the seeded x^j equal x_0 + V (V^dag M V)^{-1} V^dag r_0^j solved densely.
  * k = 1 (full reorthogonalisation) gives that Galerkin solution to rounding.
  * Linearity in the right-hand side; a duplicated right-hand side is seeded to x^1.
  * CG reaches the dense Cholesky solution.
"""
import math

import numpy as np
import pytest

from oracle import seedcg as sc
from oracle.wilson import WilsonEO, dense, flat, matvec_M
from synth.configs import CONFIGS, make_inputs
from synth.links import random_su3_links


@pytest.fixture(scope="module")
def c1():
    """The 4^4 workload at lambda_min/lambda_max ~ 1e-3, where Lanczos loses orthogonality."""
    U, phi, kappa = make_inputs("c1")
    op = WilsonEO(U, (4, 4, 4, 4), kappa)
    mv = matvec_M(op)
    B = flat(op.apply_Adag(phi))
    return op, mv, B


@pytest.fixture(scope="module")
def small():
    U, phi, kappa = make_inputs("t4")
    op = WilsonEO(U, (4, 4, 4, 4), kappa)
    mv = matvec_M(op)
    B = flat(op.apply_Adag(phi))
    return op, mv, B


def test_lu_of_T_eq2(small):
    op, mv, B = small
    out = sc.seed_cg(mv, B[:1], k=0, tol=1e-10, m=30)
    a, b, d, g = out["alpha"], out["beta"], out["delta"], out["gamma"]
    m = len(a)
    T = sc.tridiag(a, b)
    L = np.eye(m) + np.diag(g[1:m], -1)
    Umat = np.diag(d) + np.diag(b[1:m], 1)
    assert np.max(np.abs(L @ Umat - T)) < 1e-13 * np.max(np.abs(T))


def test_T_from_cg_coefficients(small):
    op, mv, B = small
    n = 40
    out = sc.seed_cg(mv, B[:1], k=0, tol=1e-10, m=n)
    acg, bcg, _ = sc.cg_coefficients(mv, B[0], n)
    alpha_T = np.empty(n)
    alpha_T[0] = 1.0 / acg[0]
    alpha_T[1:] = 1.0 / acg[1:] + bcg[:-1] / acg[:-1]
    beta_T = np.sqrt(bcg[:-1]) / acg[:-1]
    assert np.max(np.abs(out["alpha"] - alpha_T) / np.abs(alpha_T)) < 1e-11
    assert np.max(np.abs(out["beta"][1:n] - beta_T) / beta_T) < 1e-11


def test_dlanczos_iterate_is_cg_iterate_and_estimate(small):
    op, mv, B = small
    b = B[0]
    bn = np.linalg.norm(b)
    for i in (1, 2, 7, 25, 60):
        out = sc.seed_cg(mv, B[:1], k=0, tol=1e-10, m=i)
        x_cg = np.zeros_like(b)
        r = b.copy()
        p = r.copy()
        rr = np.vdot(r, r).real
        for _ in range(i):
            q = mv(p)
            a = rr / np.vdot(p, q).real
            x_cg += a * p
            r -= a * q
            rn = np.vdot(r, r).real
            p = r + (rn / rr) * p
            rr = rn
        assert np.linalg.norm(out["X"][0] - x_cg) <= 1e-10 * np.linalg.norm(x_cg)
        true = np.linalg.norm(b - mv(out["X"][0])) / bn
        assert abs(out["est"][-1] - true) <= 1e-6 * true + 1e-13


def test_galerkin_identity_eq1(c1):
    op, mv, B = c1
    out = sc.seed_cg(mv, B, k=10, tol=1e-10, past=1.5)
    assert out["status"] == "ok" and out["i_conv"] is not None
    assert out["m"] == math.ceil(1.5 * out["i_conv"])
    Xg = sc.galerkin(mv, out["V"], out["R0"])
    rel = np.linalg.norm(out["X"] - Xg, axis=1) / np.linalg.norm(Xg, axis=1)
    assert np.max(rel) < 1e-7, rel
    assert sc.orth_loss(out["V"]) < 1e-8


def test_full_reorth_k1_is_exact_galerkin(small):
    op, mv, B = small
    out = sc.seed_cg(mv, B, k=1, tol=1e-10, m=80)
    assert sc.orth_loss(out["V"]) < 1e-13
    Xg = sc.galerkin(mv, out["V"], out["R0"])
    rel = np.linalg.norm(out["X"] - Xg, axis=1) / np.linalg.norm(Xg, axis=1)
    assert np.max(rel) < 1e-11, rel


def test_no_reorth_loses_orthogonality_past_convergence(c1):
    op, mv, B = c1
    plain = sc.seed_cg(mv, B[:1], k=0, tol=1e-10, past=1.5)
    po = sc.seed_cg(mv, B[:1], k=10, tol=1e-10, past=1.5)
    assert sc.orth_loss(po["V"]) < 1e-8
    assert sc.orth_loss(plain["V"]) > 1e3 * sc.orth_loss(po["V"])


def test_linearity_and_duplicate_rhs(small):
    op, mv, B = small
    a, c = 0.7 - 0.2j, -1.3 + 0.4j
    Bl = np.stack([B[0], B[1], B[2], a * B[1] + c * B[2], B[0]])
    out = sc.seed_cg(mv, Bl, k=10, tol=1e-10, past=1.5)
    X = out["X"]
    comb = a * X[1] + c * X[2]
    assert np.linalg.norm(X[3] - comb) <= 1e-12 * np.linalg.norm(comb)
    # a duplicate of b^1 is seeded to the RHS-1 iterate (exact up to the orthogonality loss)
    assert np.linalg.norm(X[4] - X[0]) <= 1e-7 * np.linalg.norm(X[0])


def test_seeded_residuals_and_cg_finish(c1):
    op, mv, B = c1
    out = sc.seed_cg(mv, B, k=10, tol=1e-10, past=1.5)
    res0 = sc.true_relres(mv, B, np.zeros_like(B))
    res = sc.true_relres(mv, B, out["X"])
    assert res[0] < 1e-10
    assert np.all(res[1:] < res0[1:])
    # the seeded guesses converge in fewer CG iterations than a cold start
    for j in range(1, B.shape[0]):
        _, it_seed, r_seed, _ = sc.cg(mv, B[j], out["X"][j], tol=1e-10)
        _, it_cold, r_cold, _ = sc.cg(mv, B[j], None, tol=1e-10)
        assert r_seed <= 1e-10 and r_cold <= 1e-10
        assert it_seed < it_cold


def test_cg_matches_dense_cholesky():
    dims = (4, 2, 2, 4)
    rng = np.random.default_rng(3)
    U = random_su3_links(dims, 0.6, rng)
    op = WilsonEO(U, dims, 0.14)
    mv = matvec_M(op)
    n = 12 * op.Vh
    M = dense(mv, n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    L = np.linalg.cholesky(0.5 * (M + M.conj().T))
    x_ref = np.linalg.solve(L.conj().T, np.linalg.solve(L, b))
    x, it, res, _ = sc.cg(mv, b, tol=1e-12)
    assert res <= 1e-12
    cond = np.linalg.cond(M)
    assert np.linalg.norm(x - x_ref) <= 10 * cond * 1e-12 * np.linalg.norm(x_ref)


def test_breakdown_on_few_distinct_eigenvalues():
    """Unit links on 2^4: M has few distinct eigenvalues, so Lanczos ends in an invariant subspace."""
    dims = (2, 2, 2, 2)
    V = 16
    U = np.tile(np.eye(3, dtype=np.complex128), (4, V, 1, 1))
    op = WilsonEO(U, dims, 0.1)
    mv = matvec_M(op)
    rng = np.random.default_rng(1)
    B = rng.standard_normal((2, 96)) + 1j * rng.standard_normal((2, 96))
    n_distinct = len(np.unique(np.round(np.linalg.eigvalsh(dense(mv, 96)), 10)))
    out = sc.seed_cg(mv, B, k=0, tol=1e-30, past=1.5, m_max=200)
    assert out["status"] == "breakdown"
    assert out["m"] <= n_distinct
    assert sc.true_relres(mv, B[:1], out["X"][:1])[0] < 1e-12


def test_repeated_seeding_pins(c1):
    """Repeated seeding: one system is Algorithm 1 run to convergence then CG; after run j the
    residual of system j+1 is orthogonal to run j's basis (the Galerkin condition of Eq. (1)); every
    final solution meets the FP64 tolerance."""
    op, mv, B = c1
    one = sc.repeated_seed(mv, B[:1], k=10, tol=1e-10)
    ref = sc.seed_cg(mv, B[:1], k=10, tol=1e-10, past=1.0)
    assert one["lanczos"] == [ref["m"]]
    out = sc.repeated_seed(mv, B, k=10, tol=1e-10)
    for j, r in enumerate(out["seeded"]):
        V = out["bases"][j]
        assert np.max(np.abs(V.conj() @ r)) <= 1e-8 * np.linalg.norm(B[j + 1])
    res = sc.true_relres(mv, B, out["X"])
    assert np.all(res <= 1e-10)


def _flux_case(flux):
    from dataclasses import replace

    from synth.configs import make_links, make_sources
    cfg = replace(CONFIGS["c1"], flux=flux)
    op = WilsonEO(make_links(cfg), cfg.dims, 0.17)
    mv = matvec_M(op)
    return mv, flat(op.apply_Adag(make_sources(cfg)))


def test_seeding_pays_only_with_isolated_low_modes():
    """The gain of the seeded guesses comes from the low modes that the first system's Krylov space
    resolves.  On 4^4 with one flux quantum through two planes the operator has near-zero modes
    apart from its bulk (lambda_min/lambda_max ~ 4e-5 at kappa 0.17), and the seeded systems need at
    most 0.35x the cold-start CG iterations (35 against 134); on the same links without the flux
    the low spectrum is dense and the seeded systems need at least 0.9x (46 against 46)."""
    for flux, lo, hi in (((1, 1), 0.0, 0.35), (None, 0.9, 1.0)):
        mv, B = _flux_case(flux)
        out = sc.seed_cg(mv, B, k=10, tol=1e-10, past=1.5)
        for j in range(1, B.shape[0]):
            _, it_s, r_s, _ = sc.cg(mv, B[j], out["X"][j], tol=1e-10)
            _, it_c, r_c, _ = sc.cg(mv, B[j], None, tol=1e-10)
            assert r_s <= 1e-10 and r_c <= 1e-10
            assert lo <= it_s / it_c <= hi, (flux, j, it_s, it_c)


def test_reorthogonalising_against_fp32_roundings_keeps_the_seeding_gain():
    """8^4 with one flux quantum through two planes (kappa 0.14, near-zero modes apart from the bulk),
    six point sources, k = 10: Algorithm 1 with its periodic reorthogonalisation projecting against
    the FP32 roundings of the basis vectors (the stored basis, the recurrence and the seeding in FP64)
    stops at the same m, leaves the basis orthogonal to FP32 rounding only, and its seeded guesses
    need the same CG iterations (within 1) as those of the FP64 reorthogonalisation."""
    from synth.configs import make_links, with_changes
    from synth.sources import point_sources
    dims = (8, 8, 8, 8)
    U = make_links(with_changes(CONFIGS["c5"], dims=dims, flux=(1, 1)))
    op = WilsonEO(U, dims, 0.14)
    B = flat(op.apply_Adag(point_sources(dims, 6)))
    mv = matvec_M(op)
    rnd = lambda Q: Q.astype(np.complex64).astype(np.complex128)
    runs = [sc.seed_cg(mv, B, k=10, tol=1e-10, past=1.5), sc.seed_cg(mv, B, k=10, tol=1e-10, past=1.5, reorth_basis=rnd)]
    assert runs[0]["m"] == runs[1]["m"]
    assert sc.orth_loss(runs[0]["V"]) <= 1e-13 and 1e-12 < sc.orth_loss(runs[1]["V"]) <= 1e-6
    its = [np.array([sc.cg(mv, B[j], r["X"][j], tol=1e-10)[1] for j in range(1, 6)]) for r in runs]
    assert np.max(np.abs(its[0] - its[1])) <= 1, its
