"""Pins of the oracle's deflated CG (oracle/deflation.py), CPU only.

  * no deflation vectors: deflated CG is plain CG, iterate for iterate;
  * any W (here random, not an invariant subspace): W^dag r_j = 0 and W^dag M p_j = 0 at every
    iteration (the defining properties of the method; a sign, a conjugation or a transposed
    operand in mu breaks them), and the solution is the dense solve's;
  * W = the exact lowest eigenvectors of M: fewer iterations than plain CG;
  * Ritz pairs of a full Lanczos run (reorthogonalised at every step) are the eigenpairs of M.
"""
import numpy as np
import pytest

from oracle import deflation as dfl
from oracle import seedcg as sc
from oracle.wilson import WilsonEO, dense, flat, matvec_M
from synth.links import random_su3_links

DIMS = (4, 2, 2, 4)


@pytest.fixture(scope="module")
def system():
    U = random_su3_links(DIMS, 0.5, np.random.default_rng(41))
    op = WilsonEO(U, DIMS, 0.16)
    mv = matvec_M(op)
    N = 12 * op.Vh
    Md = dense(mv, N)
    Md = 0.5 * (Md + Md.conj().T)
    rng = np.random.default_rng(42)
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return dict(mv=mv, N=N, M=Md, b=b, rng=rng)


def test_without_deflation_vectors_it_is_cg(system):
    mv, b = system["mv"], system["b"]
    x1, it1, res1 = dfl.deflated_cg(mv, b, None, [], tol=1e-10)
    x2, it2, res2, _ = sc.cg(mv, b, None, tol=1e-10)
    assert it1 == it2
    assert np.linalg.norm(x1 - x2) <= 1e-13 * np.linalg.norm(x2)


def test_invariants_and_solution_with_random_w(system):
    mv, b, M, N = system["mv"], system["b"], system["M"], system["N"]
    W = system["rng"].standard_normal((5, N)) + 1j * system["rng"].standard_normal((5, N))
    x, it, res, hist = dfl.deflated_cg(mv, b, None, W, tol=1e-10, history=True)
    assert res <= 1e-10 and it > 5
    # both hold to rounding, measured against the sizes at the start of the iteration
    wn = np.linalg.norm(W, axis=1)
    r_scale = np.linalg.norm(hist[0][0])
    mp_scale = max(np.linalg.norm(M @ p) for _, p in hist)
    for r, p in hist:
        assert np.max(np.abs(W.conj() @ r) / wn) <= 1e-11 * r_scale
        assert np.max(np.abs(W.conj() @ (M @ p)) / wn) <= 1e-11 * mp_scale
    xs = np.linalg.solve(M, b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_exact_low_eigenvectors_cut_the_iterations(system):
    mv, b, M = system["mv"], system["b"], system["M"]
    lam, Q = np.linalg.eigh(M)
    W = Q[:, :12].T
    _, it_d, res_d = dfl.deflated_cg(mv, b, None, W, tol=1e-10)
    _, it_c, _, _ = sc.cg(mv, b, None, tol=1e-10)
    assert res_d <= 1e-10
    assert it_d < 0.8 * it_c, (it_d, it_c)


def test_ritz_pairs_of_a_lanczos_run(system):
    """Lanczos reorthogonalised at every step, 120 steps: the lowest two Ritz pairs have converged to
    eigenpairs of M; every Ritz value lies above the eigenvalue of the same index (interlacing)."""
    mv, b, M, N = system["mv"], system["b"], system["M"], system["N"]
    ref = sc.seed_cg(mv, b[None, :], k=1, tol=1e-300, past=0.0, m=120)
    theta, U = dfl.ritz(ref["V"], ref["alpha"], ref["beta"], 4)
    lam = np.linalg.eigvalsh(M)
    assert np.all(np.abs(theta[:2] - lam[:2]) <= 1e-8 * lam[-1]), (theta, lam[:4])
    assert np.all(theta >= lam[:4] - 1e-10 * lam[-1])
    for t, u in zip(theta[:2], U[:2]):
        assert abs(np.linalg.norm(u) - 1.0) <= 1e-10
        assert np.linalg.norm(M @ u - t * u) <= 1e-4 * lam[-1]   # vectors converge linearly, values quadratically


def test_deflation_pays_with_isolated_low_modes():
    """8 Ritz vectors of a Seed-CG run (k = 10, past 1.5) deflate plain CG from zero. On 4^4 with the
    flux background at kappa 0.16 (six near-zero modes apart from the bulk) that halves CG (at most
    0.6x: about 51 against 107); on the same links without the flux it saves little (at least
    0.85x: about 47 against 50)."""
    from dataclasses import replace

    from oracle.wilson import WilsonEO, flat, matvec_M
    from synth.configs import CONFIGS, make_links, make_sources
    for flux, lo, hi in (((1, 1), 0.0, 0.6), (None, 0.85, 1.0)):
        cfg = replace(CONFIGS["c1"], flux=flux)
        op = WilsonEO(make_links(cfg), cfg.dims, 0.16)
        mv = matvec_M(op)
        B = flat(op.apply_Adag(make_sources(cfg)))
        ref = sc.seed_cg(mv, B, k=10, tol=1e-10, past=1.5)
        _, W = dfl.ritz(ref["V"], ref["alpha"], ref["beta"], 8)
        for j in (1, 3):
            _, it_d, r_d = dfl.deflated_cg(mv, B[j], None, W, tol=1e-10)
            _, it_c, r_c, _ = sc.cg(mv, B[j], None, tol=1e-10)
            assert r_d <= 1e-10 and r_c <= 1e-10
            assert lo <= it_d / it_c <= hi, (flux, j, it_d, it_c)


def _hpd_precond(system):
    """An HPD preconditioner independent of the method: a random well-conditioned HPD matrix."""
    rng = np.random.default_rng(43)
    N = system["N"]
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    d = rng.uniform(0.5, 2.0, N)
    P = (Q * d) @ Q.conj().T
    return 0.5 * (P + P.conj().T)


def test_preconditioned_invariants_and_solution(system):
    """Deflated PCG keeps W^dag r_j = 0 and W^dag M p_j = 0 and solves the system."""
    mv, b, M, N = system["mv"], system["b"], system["M"], system["N"]
    P = _hpd_precond(system)
    W = system["rng"].standard_normal((5, N)) + 1j * system["rng"].standard_normal((5, N))
    x, it, res, hist = dfl.deflated_cg(mv, b, None, W, tol=1e-10, history=True, precond=lambda r: P @ r)
    assert res <= 1e-10 and it > 5
    wn = np.linalg.norm(W, axis=1)
    r_scale = np.linalg.norm(hist[0][0])
    mp_scale = max(np.linalg.norm(M @ p) for _, p in hist)
    for r, p in hist:
        assert np.max(np.abs(W.conj() @ r) / wn) <= 1e-11 * r_scale
        assert np.max(np.abs(W.conj() @ (M @ p)) / wn) <= 1e-11 * mp_scale
    xs = np.linalg.solve(M, b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_preconditioned_form_is_scale_invariant_and_reduces_to_pcg(system):
    """P = c I gives deflated CG's iterates; without W it is the oracle's plain PCG."""
    from oracle import learned as lk
    mv, b, N = system["mv"], system["b"], system["N"]
    W = system["rng"].standard_normal((3, N)) + 1j * system["rng"].standard_normal((3, N))
    x1, it1, _ = dfl.deflated_cg(mv, b, None, W, tol=1e-10)
    x2, it2, _ = dfl.deflated_cg(mv, b, None, W, tol=1e-10, precond=lambda r: 3.0 * r)
    assert it1 == it2 and np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x1)
    P = _hpd_precond(system)
    x3, it3, _ = dfl.deflated_cg(mv, b, None, [], tol=1e-10, precond=lambda r: P @ r)
    x4, it4 = lk.pcg(mv, lambda r: P @ r, b, None, tol=1e-10)
    assert it3 == it4 and np.linalg.norm(x3 - x4) <= 1e-12 * np.linalg.norm(x4)
