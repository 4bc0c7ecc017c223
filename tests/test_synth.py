"""Input generators: SU(3) links, APE smearing, sources, reproducibility (CPU only)."""
import numpy as np

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
