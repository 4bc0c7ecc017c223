"""Failure paths and report fields of the C ABI on small lattices (one GPU).

  * SEEDCG_ERR_NOCONV: solve_rest stopped by max_iter returns the status, leaves its last iterate
    in X and reports that iterate's FP64 true residual (checked by the oracle's M).
  * A non-finite right-hand side or starting guess is refused with SEEDCG_ERR_ARG before any
    iteration, and the handle solves the next clean system normally.
  * Deflated CG keeps its deflation space after release_basis (the Ritz vectors are built before
    the basis goes), and refuses more than 24 right-hand sides.
  * Report fields: the Lanczos estimate of RHS 1 meets tol at m, the orthogonality-loss figure is 0
    without reorthogonalisation and small with it, the CG estimates meet tol.
"""
import math

import numpy as np
import pytest

from gpu_helpers import cuda, host, print_case
from oracle import seedcg as osc
from oracle.wilson import WilsonEO, flat, matvec_M
from synth.configs import make_inputs

pytestmark = pytest.mark.gpu


def _problem(name="t8", nrhs=None):
    U, phi, kappa = make_inputs(name)
    dims = {"t4": (4, 4, 4, 4), "t8": (8, 8, 8, 8), "c1": (4, 4, 4, 4)}[name]
    op = WilsonEO(U, dims, kappa)
    B = op.apply_Adag(phi if nrhs is None else phi[:nrhs])
    return U, dims, kappa, op, B


def _solver(U, dims, kappa, **kw):
    from paper_0901_3512_amd import SeedCG
    return SeedCG(cuda(U), dims, kappa, **kw)


def test_noconv_returns_last_iterate_and_its_residual():
    print_case("noconv t8 max_iter=7")
    U, dims, kappa, op, B = _problem("t8")
    s = _solver(U, dims, kappa, max_iter=7)
    X = cuda(np.zeros_like(B))
    X, rep = s.solve_rest(cuda(B), X, raise_on_noconv=False)
    assert rep["status"] == "ERR_NOCONV"
    assert all(it <= 7 + 1 for it in rep["iters"])
    res = osc.true_relres(matvec_M(op), flat(B), flat(host(X)))
    got = np.array(rep["true_relres"])
    assert np.all(got > 1e-10) and np.all(res < 1.0)         # moved from x0 = 0, not converged
    assert np.allclose(got, res, rtol=1e-8, atol=0), (got, res)
    from paper_0901_3512_amd import SeedCGError
    with pytest.raises(SeedCGError) as e:
        s.solve_rest(cuda(B), X)
    assert e.value.code == -5


@pytest.mark.parametrize("where", ["B", "X"])
def test_non_finite_input_is_refused_then_handle_recovers(where):
    from paper_0901_3512_amd import SeedCGError
    print_case("non-finite", where)
    U, dims, kappa, op, B = _problem("t4")
    s = _solver(U, dims, kappa, reorth_k=10)
    bad_B = B.copy()
    bad_X = np.zeros_like(B)
    if where == "B":
        bad_B[1, 5, 2, 1] = np.nan
    else:
        bad_X[2, 0, 0, 0] = np.inf
    for call in ("seed", "rest"):
        with pytest.raises(SeedCGError) as e:
            if call == "seed":
                s.solve_seed(cuda(bad_B), cuda(bad_X))
            else:
                s.solve_rest(cuda(bad_B), cuda(bad_X))
        assert e.value.code == -1 and "non-finite" in str(e.value)
    X, _ = s.solve_seed(cuda(B))
    X, rep = s.solve_rest(cuda(B), X)
    assert max(rep["true_relres"]) <= 1e-10
    assert np.all(osc.true_relres(matvec_M(op), flat(B), flat(host(X))) <= 1e-10)


def test_deflation_survives_release_basis():
    print_case("deflation after release_basis t8")
    U, dims, kappa, op, B = _problem("t8")
    s = _solver(U, dims, kappa, reorth_k=10, deflate=8)
    X, _ = s.solve_seed(cuda(B))
    X, rep1 = s.solve_rest(cuda(B), X)
    theta = s.get_ritz()
    assert len(theta) == 8
    s.release_basis()
    # new right-hand sides after the basis is gone: still deflated, still solved
    rng = np.random.default_rng(5)
    phi2 = (rng.standard_normal(B.shape) + 1j * rng.standard_normal(B.shape)) / math.sqrt(2)
    B2 = op.apply_Adag(phi2)
    X2, rep2 = s.solve_rest(cuda(B2), cuda(np.zeros_like(B2)))
    assert s.get_ritz() == theta
    res = osc.true_relres(matvec_M(op), flat(B2), flat(host(X2)))
    assert np.all(res <= 1e-10), res


def test_deflation_refuses_more_than_24_rhs():
    from paper_0901_3512_amd import SeedCGError
    print_case("deflation nrhs 25")
    U, dims, kappa, op, B = _problem("t4")
    rng = np.random.default_rng(7)
    phi = (rng.standard_normal((25,) + B.shape[1:]) + 1j * rng.standard_normal((25,) + B.shape[1:])) / math.sqrt(2)
    B25 = op.apply_Adag(phi)
    s = _solver(U, dims, kappa, reorth_k=10, deflate=4)
    X, _ = s.solve_seed(cuda(B25))
    with pytest.raises(SeedCGError) as e:
        s.solve_rest(cuda(B25), X)
    assert e.value.code == -1 and "24" in str(e.value)
    # 24 of them are fine
    X24, rep = s.solve_rest(cuda(B25[:24]), cuda(np.zeros_like(B25[:24])))
    assert max(rep["true_relres"]) <= 1e-10


def test_report_estimates_and_orthogonality_loss():
    print_case("report fields c1")
    U, dims, kappa, op, B = _problem("c1")
    tol = 1e-10
    for k in (0, 1, 10):
        s = _solver(U, dims, kappa, reorth_k=k, tol=tol)
        X, rs = s.solve_seed(cuda(B))
        assert rs["est_relres"][0] <= tol * 1.0000001
        assert all(math.isnan(e) for e in rs["est_relres"][1:])
        if k == 0:
            assert rs["orth_loss_max"] == 0.0
        elif k == 1:
            assert 0.0 < rs["orth_loss_max"] <= 1e-12      # full reorthogonalisation keeps it at rounding
        else:
            assert 1e-16 < rs["orth_loss_max"] <= 1e-3      # it grows between passes, as Lanczos does
        X, rr = s.solve_rest(cuda(B), X)
        assert all(e <= tol for e in rr["est_relres"])
        assert max(rr["true_relres"]) <= tol
