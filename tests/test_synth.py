"""Input generators: SU(3) links, APE smearing, sources, reproducibility (CPU only)."""
import numpy as np
import pytest

from synth import ape_smear, gaussian_sources, plaquette, point_sources, random_su3_links, z2_sources
from synth.configs import CONFIGS, batch_members, make_inputs


def _su3_errors(U):
    U = U.reshape(-1, 3, 3)
    unit = np.max(np.abs(np.conj(np.swapaxes(U, -1, -2)) @ U - np.eye(3)))
    det = np.max(np.abs(np.linalg.det(U) - 1.0))
    return unit, det


def test_links_are_su3_and_reproducible():
    dims = (4, 2, 2, 4)
    U = random_su3_links(dims, 0.5, np.random.default_rng([1, 0]))
    u, d = _su3_errors(U)
    assert u < 1e-14 and d < 1e-14
    U2 = random_su3_links(dims, 0.5, np.random.default_rng([1, 0]))
    assert np.array_equal(U, U2)


def test_ape_smearing_stays_su3_and_raises_plaquette():
    dims = (4, 4, 4, 4)
    U = random_su3_links(dims, 0.5, np.random.default_rng(2))
    S = ape_smear(U, dims, 0.5, 2)
    u, d = _su3_errors(S)
    assert u < 1e-13 and d < 1e-13
    assert plaquette(S, dims) > plaquette(U, dims)
    # the unit gauge field is a fixed point of smearing
    one = np.tile(np.eye(3, dtype=np.complex128), (4, 256, 1, 1))
    assert np.max(np.abs(ape_smear(one, dims, 0.5, 1) - one)) < 1e-14


def test_sources():
    dims = (4, 4, 4, 4)
    P = point_sources(dims, 12)
    assert P.shape == (12, 128, 4, 3)
    for j in range(12):
        s, c = divmod(j, 3)
        assert P[j, 0, s, c] == 1 and np.count_nonzero(P[j]) == 1
    Z = z2_sources(dims, 3, np.random.default_rng(0))
    assert set(np.unique(Z.real)) == {-1.0, 1.0} and np.all(Z.imag == 0)
    G = gaussian_sources(dims, 2, np.random.default_rng(0))
    assert abs(np.mean(np.abs(G) ** 2) - 1.0) < 0.1


def test_workloads():
    assert CONFIGS["c2"].nrhs == 12 and CONFIGS["c3"].nrhs == 24
    m = batch_members()
    assert len(m) == 64
    assert {c.dims for c in m} == {(8, 8, 8, 8), (8, 8, 8, 16), (12, 12, 12, 24), (12, 12, 12, 12)}
    assert all(1e-4 <= c.ratio <= 1e-3 for c in m)
    U, phi, kappa = make_inputs("c1")
    assert phi.shape == (4, 128, 4, 3) and 0.7 < kappa < 0.9


def test_flux_background_plaquettes_and_flux_quanta():
    """Every (x, y) plaquette carries 2 pi n01 / (Lx Ly) per unit charge and every (z, t) one
    2 pi n23 / (Lz Lt), the wrapped ones included; the other planes carry none; so each (x, y)
    slice holds exactly n01 flux quanta and each (z, t) slice n23.  Links are special unitary."""
    from synth.links import _as5, _axis, _dag, flux_background
    dims = (4, 6, 4, 8)
    n01, n23 = 1, 2
    U = flux_background(dims, n01, n23)
    eye = np.eye(3)
    assert np.allclose(U @ _dag(U), eye, atol=1e-14)
    assert np.allclose(np.linalg.det(U), 1.0, atol=1e-14)
    U5 = _as5(U, dims)
    want = {(0, 1): 2 * np.pi * n01 / (4 * 6), (2, 3): 2 * np.pi * n23 / (4 * 8)}
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = (U5[mu] @ np.roll(U5[nu], -1, axis=_axis(mu)) @ _dag(np.roll(U5[mu], -1, axis=_axis(nu)))
                 @ _dag(U5[nu]))
            th = want.get((mu, nu), 0.0)
            for c, q in enumerate((1, 1, -2)):
                assert np.allclose(P[..., c, c], np.exp(1j * q * th), atol=1e-12), (mu, nu, c)
            assert np.allclose(P * (1 - np.eye(3)), 0, atol=1e-14)   # diagonal: an abelian field
    # flux quanta per slice: the plaquette angles of colour 0 summed over one (x, y) slice
    P01 = (U5[0] @ np.roll(U5[1], -1, axis=_axis(0)) @ _dag(np.roll(U5[0], -1, axis=_axis(1))) @ _dag(U5[1]))
    assert abs(np.angle(P01[0, 0, :, :, 0, 0]).sum() / (2 * np.pi) - n01) < 1e-12


def test_flux_background_workload_keeps_the_base_links_and_charges_must_cancel():
    from dataclasses import replace

    from synth.configs import make_links
    from synth.links import flux_background
    base = make_links(CONFIGS["c1"])
    with_flux = make_links(replace(CONFIGS["c1"], flux=(1, 1)))
    assert np.allclose(with_flux, flux_background((4, 4, 4, 4), 1, 1) @ base, atol=0)
    with pytest.raises(ValueError):
        flux_background((4, 4, 4, 4), 1, 1, charges=(1, 1, 1))


def test_flux_background_gives_the_index_theorem_count_of_near_zero_modes():
    """One flux quantum through the (x, y) and the (z, t) planes carries topological charge
    q^2 n01 n23 for a colour of charge q, so the charges (1, 1, -2) give 1 + 1 + 4 = 6 would-be
    zero modes.  On 4^4 near the critical kappa (0.16) the oracle's dense M has exactly six
    eigenvalues below 1% of lambda_max, and a gap of more than 4x above them; the same links
    without the flux have a dense low spectrum (the ten lowest within 30% of each other)."""
    from dataclasses import replace

    from oracle.wilson import WilsonEO, dense, matvec_M
    from synth.configs import make_links
    for flux in ((1, 1), None):
        cfg = replace(CONFIGS["c1"], flux=flux)
        op = WilsonEO(make_links(cfg), cfg.dims, 0.16)
        M = dense(matvec_M(op), 12 * op.Vh)
        lam = np.linalg.eigvalsh(0.5 * (M + M.conj().T))
        rel = lam / lam[-1]
        if flux:
            assert np.sum(rel < 1e-2) == 6, rel[:10]
            assert lam[6] / lam[5] > 4.0, rel[:10]
        else:
            assert lam[9] / lam[0] < 1.3, rel[:10]


def test_stored_kappas_of_the_16x32_workloads():
    """The oracle's search records (synth/kappa.json): on the named 16^3 x 32 links the ratio 1e-5
    is unreachable (the minimum, ~9e-4, is kept); on the same links with the flux background the
    search reaches it within its 0.05-decade tolerance, at a kappa just above the other's minimum."""
    import json
    import math
    import os

    import synth
    tab = json.load(open(os.path.join(os.path.dirname(synth.__file__), "kappa.json")))
    c2, c2t = tab["c2"], tab["c2t"]
    assert c2["target_unreachable"] and 5e-4 < c2["ratio"] < 2e-3
    assert not c2t["target_unreachable"] and abs(math.log10(c2t["ratio"] / 1e-5)) <= 0.05
    assert abs(c2t["kappa"] - c2["kappa"]) < 0.005
