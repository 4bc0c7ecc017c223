"""Pins of the oracle's learned preconditioner (CPU only).

K = identity at initialisation; T_{+mu}^dag = T_{-mu}; K^dag is the adjoint of K; K K^dag is
Hermitian positive semi-definite (dense, small lattice); gauge covariance; the hand-derived
Wirtinger gradient against central finite differences; Adam's first step; PCG with P = 1 is CG.
"""
import numpy as np
import pytest

from oracle import learned as lk
from oracle import seedcg as sc
from oracle.wilson import WilsonEO, flat, matvec_M
from synth.links import random_su3_links

DIMS = (4, 2, 2, 4)


@pytest.fixture(scope="module")
def lat():
    U = random_su3_links(DIMS, 0.6, np.random.default_rng(21))
    return lk.Lattice(U, DIMS), U


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _randW(rng, scale=0.3):
    W = lk.identity_weights() + scale * _rand(rng, lk.NLAYER, lk.NDIR, 4, 4)
    return W


def test_identity_initialisation(lat):
    L, _ = lat
    rng = np.random.default_rng(0)
    x = _rand(rng, 2, L.V // 2, 4, 3)
    W = lk.identity_weights()
    assert np.max(np.abs(lk.apply_K(L, W, x) - x)) == 0
    assert np.max(np.abs(lk.apply_P(L, W, x) - x)) == 0


def test_transport_adjoints(lat):
    L, _ = lat
    rng = np.random.default_rng(1)
    psi = _rand(rng, L.V, 4, 3)
    phi = _rand(rng, L.V, 4, 3)
    for d in range(1, 9):
        lhs = np.vdot(phi, L.transport(psi, d))
        rhs = np.vdot(L.transport(phi, lk.adjoint_dir(d)), psi)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_Kdag_is_adjoint_and_P_is_hpsd(lat):
    L, _ = lat
    rng = np.random.default_rng(2)
    W = _randW(rng)
    Vh = L.V // 2
    x = _rand(rng, Vh, 4, 3)
    y = _rand(rng, Vh, 4, 3)
    lhs = np.vdot(x, lk.apply_K(L, W, y))
    rhs = np.vdot(lk.apply_Kdag(L, W, x), y)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    n = 12 * Vh
    P = np.stack([flat(lk.apply_P(L, W, e.reshape(Vh, 4, 3))) for e in np.eye(n, dtype=np.complex128)]).T
    assert np.max(np.abs(P - P.conj().T)) <= 1e-12 * np.max(np.abs(P))
    assert np.linalg.eigvalsh(0.5 * (P + P.conj().T)).min() >= -1e-10 * np.max(np.abs(P))


def test_gauge_covariance(lat):
    L, U = lat
    rng = np.random.default_rng(3)
    Om = random_su3_links(DIMS, 2.0, rng)[0]
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[mu] = Om @ U[mu] @ np.conj(np.swapaxes(Om[L.fwd[mu]], -1, -2))
    Lg = lk.Lattice(Ug, DIMS)
    W = _randW(rng)
    x = _rand(rng, L.V // 2, 4, 3)
    Om_e = Om[L.even]
    rot = lambda v: np.einsum("sab,sib->sia", Om_e, v)
    assert np.max(np.abs(lk.apply_P(Lg, W, rot(x)) - rot(lk.apply_P(L, W, x)))) <= 1e-12 * np.max(np.abs(x)) * 50


def test_gradient_matches_finite_differences(lat):
    L, U = lat
    rng = np.random.default_rng(4)
    W = _randW(rng, 0.2)
    op = WilsonEO(U, DIMS, 0.12)
    Uv = _rand(rng, 2, L.V // 2, 4, 3)
    Y = op.apply_M(Uv)
    G = lk.grad(L, W, Y, Uv)
    h = 1e-6
    for (l, d, a, b) in [(0, 0, 0, 0), (0, 3, 1, 2), (1, 5, 3, 0), (2, 8, 2, 2), (2, 0, 1, 3), (1, 4, 0, 1)]:
        for part in (1.0, 1j):
            Wp = W.copy()
            Wm = W.copy()
            Wp[l, d, a, b] += h * part
            Wm[l, d, a, b] -= h * part
            fd = (lk.loss(L, Wp, Y, Uv) - lk.loss(L, Wm, Y, Uv)) / (2 * h)
            an = 2.0 * (G[l, d, a, b].real if part == 1.0 else G[l, d, a, b].imag)
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (l, d, a, b, part, fd, an)


def test_adam_first_step():
    W = lk.identity_weights()
    G = np.zeros_like(W)
    G[0, 1, 0, 0] = 0.5 - 0.25j
    st = {}
    W1 = lk.adam_step(W, G, st, lr=1e-2)
    # first step: m_hat = g, v_hat = g^2, so every real moves by lr * g / (|g| + eps)
    assert abs(W1[0, 1, 0, 0] - (-1e-2 + 1e-2j)) <= 1e-9
    assert np.max(np.abs(np.delete((W1 - W).ravel(), np.ravel_multi_index((0, 1, 0, 0), W.shape)))) == 0


def test_pcg_with_identity_is_cg(lat):
    L, U = lat
    op = WilsonEO(U, DIMS, 0.12)
    mv = matvec_M(op)
    rng = np.random.default_rng(5)
    b = flat(_rand(rng, L.V // 2, 4, 3))
    W = lk.identity_weights()
    prec = lambda r: flat(lk.apply_P(L, W, r.reshape(L.V // 2, 4, 3)))
    x1, it1 = lk.pcg(mv, prec, b, tol=1e-10)
    x2, it2, _, _ = sc.cg(mv, b, tol=1e-10)
    assert it1 == it2
    assert np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x2)


def test_neumann_start_is_first_order_inverse_of_A(lat):
    """K at the training start equals 1 + kappa^2 H_eo H_oe built by the oracle's C hop (a separate
    implementation of the transports), so A K = 1 - kappa^4 (H_eo H_oe)^2."""
    L, U = lat
    kappa = 0.13
    op = WilsonEO(U, DIMS, kappa)
    rng = np.random.default_rng(4)
    x = _rand(rng, 2, L.V // 2, 4, 3)
    ref = x + kappa ** 2 * op.H_eo(op.H_oe(x))
    got = lk.apply_K(L, lk.neumann_weights(kappa), x)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    # K^dag is the adjoint: 1 + kappa^2 (H_eo H_oe)^dag = gamma5 (1 + kappa^2 H_eo H_oe) gamma5
    from oracle.wilson import gamma5
    refd = gamma5(gamma5(x) + kappa ** 2 * op.H_eo(op.H_oe(gamma5(x))))
    gotd = lk.apply_Kdag(L, lk.neumann_weights(kappa), x)
    assert np.max(np.abs(gotd - refd)) <= 1e-13 * np.max(np.abs(refd))


def test_identity_start_is_a_saddle_for_the_hops(lat):
    """At K = 1 (all hop weights 0) the loss gradient of every hop weight is exactly zero: the only
    hop paths that reach an even site carry two hop weights.  The Neumann start has non-zero hop
    gradients."""
    L, U = lat
    op = WilsonEO(U, DIMS, 0.13)
    rng = np.random.default_rng(5)
    Uv = _rand(rng, 2, L.V // 2, 4, 3)
    Y = op.apply_M(Uv)
    G = lk.grad(L, lk.identity_weights(), Y, Uv)
    assert np.max(np.abs(G[:, 1:])) == 0.0
    assert np.max(np.abs(G[:, 0])) > 0.0
    Gn = lk.grad(L, lk.neumann_weights(0.13), Y, Uv)
    assert np.min(np.max(np.abs(Gn[:, 1:]), axis=(2, 3))) > 0.0


def test_band_loss_gradient_matches_finite_differences(lat):
    """The loss on a band of t-slices and its gradient (what a training step takes) against central
    finite differences; the band covering every slice is the whole-lattice loss."""
    L, U = lat
    op = WilsonEO(U, DIMS, 0.13)
    rng = np.random.default_rng(6)
    Uv = _rand(rng, 2, L.V // 2, 4, 3)
    Y = op.apply_M(Uv)
    W = _randW(rng, 0.2)
    band = (3, 2)
    G = lk.grad(L, W, Y, Uv, band=band)
    h = 1e-6
    for (l, d, a, b) in ((0, 0, 1, 2), (1, 4, 0, 3), (2, 7, 2, 2), (1, 0, 3, 1)):
        for comp in (1.0, 1j):
            Wp = W.copy()
            Wp[l, d, a, b] += comp * h
            Wm = W.copy()
            Wm[l, d, a, b] -= comp * h
            fd = (lk.loss(L, Wp, Y, Uv, band=band) - lk.loss(L, Wm, Y, Uv, band=band)) / (2 * h)
            # dL/dRe w = 2 Re G, dL/dIm w = 2 Im G
            an = 2 * (G[l, d, a, b].real if comp == 1.0 else G[l, d, a, b].imag)
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (l, d, a, b, comp, fd, an)
    assert lk.loss(L, W, Y, Uv, band=(0, DIMS[3])) == pytest.approx(lk.loss(L, W, Y, Uv), rel=1e-14)
