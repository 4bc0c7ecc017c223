"""The learned preconditioner P = K K^dag on the GPU against the oracle (oracle/learned.py).

Bars (the GPU applies K in FP32):
  * P x and the training loss: 2e-5 relative to max |P x| / to the loss;
  * the Wirtinger gradient of the loss: 1e-4 normwise relative;
  * identity weights: P x = x to FP32 rounding; PCG then takes the iterations of plain CG;
  * a trained K lowers the loss, and PCG with it still reaches the FP64 1e-10 residual.
"""
import numpy as np
import pytest

from gpu_helpers import cuda, host, print_case, relmax
from oracle import learned as lk
from oracle import seedcg as osc
from oracle.wilson import WilsonEO, flat, matvec_M
from synth.configs import make_inputs
from synth.links import random_su3_links

pytestmark = pytest.mark.gpu


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.fixture(scope="module")
def small():
    dims = (4, 4, 2, 4)
    U = random_su3_links(dims, 0.5, np.random.default_rng(31))
    return dims, U, lk.Lattice(U, dims)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_apply_P_matches_oracle(small, prec):
    from paper_0901_3512_amd import SeedCG
    dims, U, lat = small
    print_case("apply_P", prec)
    rng = np.random.default_rng(1)
    W = lk.identity_weights() + 0.2 * _rand(rng, 3, 9, 4, 4)
    s = SeedCG(cuda(U), dims, 0.12, prec=prec)
    s.set_precond_weights(W)
    assert np.max(np.abs(s.get_precond_weights() - W)) == 0
    x = _rand(rng, 2, lat.V // 2, 4, 3)
    y = host(s.apply_P(cuda(x)))
    assert relmax(y, lk.apply_P(lat, W, x)) <= 2e-5


def test_identity_weights(small):
    from paper_0901_3512_amd import SeedCG
    dims, U, lat = small
    print_case("identity")
    s = SeedCG(cuda(U), dims, 0.12)
    s.set_precond_weights(lk.identity_weights())
    x = _rand(np.random.default_rng(2), 1, lat.V // 2, 4, 3)
    assert relmax(host(s.apply_P(cuda(x))), x) <= 1e-7


def test_loss_and_gradient_match_oracle(small):
    from paper_0901_3512_amd import SeedCG
    dims, U, lat = small
    print_case("grad")
    rng = np.random.default_rng(3)
    W = lk.identity_weights() + 0.15 * _rand(rng, 3, 9, 4, 4)
    kappa = 0.12
    op = WilsonEO(U, dims, kappa)
    Uv = _rand(rng, 3, lat.V // 2, 4, 3)
    Y = op.apply_M(Uv)
    s = SeedCG(cuda(U), dims, kappa)
    s.set_precond_weights(W)
    loss, G = s.precond_loss_grad(cuda(Uv), cuda(Y))
    ref_loss = lk.loss(lat, W, Y, Uv)
    ref_G = lk.grad(lat, W, Y, Uv)
    assert abs(loss - ref_loss) <= 2e-5 * ref_loss
    assert np.linalg.norm(G - ref_G) <= 1e-4 * np.linalg.norm(ref_G)


@pytest.fixture(scope="module")
def t8():
    U, phi, kappa = make_inputs("t8")
    dims = (8, 8, 8, 8)
    op = WilsonEO(U, dims, kappa)
    return dict(U=U, dims=dims, kappa=kappa, B=op.apply_Adag(phi), mv=matvec_M(op))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_identity_pcg_is_cg(t8, prec):
    from paper_0901_3512_amd import SeedCG
    print_case("identity pcg", prec)
    s = SeedCG(cuda(t8["U"]), t8["dims"], t8["kappa"], prec=prec)
    B = cuda(t8["B"])
    X0 = cuda(np.zeros_like(t8["B"]))
    _, plain = s.solve_rest(B, X0.clone())
    s.set_precond_weights(lk.identity_weights())
    s.use_precond(True)
    X, pcg = s.solve_rest(B, X0.clone())
    assert all(abs(a - b) <= 2 for a, b in zip(plain["iters"], pcg["iters"])), (plain["iters"], pcg["iters"])
    assert np.all(osc.true_relres(t8["mv"], flat(t8["B"]), flat(host(X))) <= 1e-10)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_training_lowers_loss_and_pcg_converges(t8, prec):
    from paper_0901_3512_amd import SeedCG
    print_case("train", prec)
    s = SeedCG(cuda(t8["U"]), t8["dims"], t8["kappa"], prec=prec, reorth_k=10)
    B = cuda(t8["B"])
    X, rs = s.solve_seed(B)
    tr = s.train_precond(steps=100, n_ritz=8, n_lanczos=8, lr=5e-3)
    assert tr["n_ritz"] >= 4 and tr["loss1"] < tr["loss0"]
    W = s.get_precond_weights()
    # the trained weights move by at most lr per Adam step in every real
    assert np.max(np.abs((W - lk.identity_weights()).real)) <= 100 * 5e-3 * 1.0001
    s.use_precond(True)
    X2, rr = s.solve_rest(B, X.clone())
    res = osc.true_relres(t8["mv"], flat(t8["B"]), flat(host(X2)))
    assert np.all(res <= 1e-10), res
    print("train", prec, tr, "pcg iters", rr["iters"])
