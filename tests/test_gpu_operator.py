"""Kernel (a): the even-odd Wilson stencil on the GPU against the oracle's plain C operator.

FP64 bar: max |gpu - oracle| <= 1e-13 * max |oracle| (different summation order only).
"""
import numpy as np
import pytest

from gpu_helpers import cuda, host, print_case, relmax
from oracle.wilson import WilsonEO
from synth.configs import CONFIGS, make_links
from synth.links import random_su3_links

pytestmark = pytest.mark.gpu

CASES = [((2, 2, 2, 2), -1, 0.5), ((4, 4, 4, 4), -1, 0.3), ((6, 4, 2, 6), 1, 0.8), ((8, 8, 8, 8), -1, 0.3),
         ((4, 6, 8, 10), -1, 0.5), ((10, 2, 4, 2), -1, 1.0), ((32, 34, 2, 2), -1, 0.5)]


def _vecs(rng, n, Vh):
    return rng.standard_normal((n, Vh, 4, 3)) + 1j * rng.standard_normal((n, Vh, 4, 3))


# vb = 4 changes only the multi-vector variants (7, 8, 9); the quad-split ones (10, 12) take one
# vector per workgroup whatever vb asks
TPS_VB = [(t, v) for v in (1, 2, 4) for t in range(1, 13) if t != 11 and (v != 4 or t in (7, 8, 9))]


@pytest.mark.parametrize("tps,vb", TPS_VB)
@pytest.mark.parametrize("dims,t_bc,eps", CASES)
def test_apply_M_matches_oracle(dims, t_bc, eps, tps, vb, monkeypatch):
    """tps: lanes per site (1, 2, 4), or two lanes per site: 3 / 5 / 6 = one / two / four directions per
    pass, 7 = links loaded once for a group of vb vectors (2 or 4), 8 = forward and backward hops on
    separate wavefronts for a group of vb vectors (1, 2 or 4), 9 = the same with the x and y neighbours
    staged in LDS (the last lattice takes three tiles of xy-rows, with halo rows), 10 = four
    wavefronts per 64 sites (forward / backward x-y / z-t hops), 12 = 10 with non-temporal link loads;
    vb: vectors per workgroup."""
    from paper_0901_3512_amd import SeedCG
    print_case("apply_M", dims, t_bc, tps, vb)
    monkeypatch.setenv("SEEDCG_TPS", str(tps))
    monkeypatch.setenv("SEEDCG_VB", str(vb))
    rng = np.random.default_rng(abs(hash((dims, t_bc))) % 2**32)
    U = random_su3_links(dims, eps, rng)
    kappa = 0.137
    op = WilsonEO(U, dims, kappa, t_bc=t_bc)
    x = _vecs(rng, 3, op.Vh)
    s = SeedCG(cuda(U), dims, kappa, t_bc=t_bc)
    y = host(s.apply_M(cuda(x)))
    assert relmax(y, op.apply_M(x)) <= 1e-13
    y1 = host(s.apply_M(cuda(x[1])))
    assert relmax(y1[0], op.apply_M(x[1])) <= 1e-13


@pytest.mark.parametrize("dims,t_bc,eps", CASES[:4])
def test_apply_A_and_Adag(dims, t_bc, eps):
    from paper_0901_3512_amd import SeedCG
    print_case("apply_A", dims, t_bc)
    rng = np.random.default_rng(7)
    U = random_su3_links(dims, eps, rng)
    kappa = 0.21
    op = WilsonEO(U, dims, kappa, t_bc=t_bc)
    x = _vecs(rng, 2, op.Vh)
    s = SeedCG(cuda(U), dims, kappa, t_bc=t_bc)
    assert relmax(host(s.apply_A(cuda(x))), op.apply_A(x)) <= 1e-13
    assert relmax(host(s.apply_A(cuda(x), dagger=True)), op.apply_Adag(x)) <= 1e-13


def test_apply_M_full_size_16x16x16x32():
    """The benchmark lattice (16^3 x 32, APE-smeared links): every output element, at the launch shape the solver uses."""
    from paper_0901_3512_amd import SeedCG
    print_case("apply_M c2 size")
    cfg = CONFIGS["c2"]
    U = make_links(cfg)
    kappa = 0.25
    op = WilsonEO(U, cfg.dims, kappa)
    rng = np.random.default_rng(3)
    x = _vecs(rng, 2, op.Vh)
    s = SeedCG(cuda(U), cfg.dims, kappa)
    y = host(s.apply_M(cuda(x)))
    assert relmax(y, op.apply_M(x)) <= 1e-13


def test_free_field_plane_wave_eigenvector():
    """Unit links, p = (0, 0, 0, pi/Lt), spinor with gamma_4 chi = chi: M psi = |1 - 4k^2 (C - iS)^2|^2 psi,
    C = 3 + cos(pi/Lt), S = sin(pi/Lt) (closed form of the free even-odd operator)."""
    from paper_0901_3512_amd import SeedCG
    print_case("plane wave")
    dims = (8, 8, 8, 16)
    Lx, Ly, Lz, Lt = dims
    V = int(np.prod(dims))
    Vh = V // 2
    U = np.tile(np.eye(3, dtype=np.complex128), (4, V, 1, 1))
    kappa = 0.12
    s = SeedCG(cuda(U), dims, kappa)
    h = np.arange(Vh)
    t = h // (Lx // 2 * Ly * Lz)
    pt = np.pi / Lt
    chi = np.array([1.0, 0.0, 1.0, 0.0]) / np.sqrt(2.0)
    psi = np.zeros((Vh, 4, 3), dtype=np.complex128)
    psi[:, :, 1] = np.exp(1j * pt * t)[:, None] * chi[None, :]
    C, S = 3.0 + np.cos(pt), np.sin(pt)
    lam = abs(1.0 - 4.0 * kappa ** 2 * (C - 1j * S) ** 2) ** 2
    y = host(s.apply_M(cuda(psi)))[0]
    assert relmax(y, lam * psi) <= 1e-13


def test_two_row_links_match_full_links(monkeypatch):
    """On a special-unitary field the stencil reads two-row links and rebuilds the third row; the
    result equals the full-link stencil to rounding (and both equal the oracle)."""
    from paper_0901_3512_amd import SeedCG
    print_case("two-row links")
    dims = (8, 4, 6, 8)
    rng = np.random.default_rng(11)
    U = random_su3_links(dims, 0.9, rng)
    op = WilsonEO(U, dims, 0.14)
    x = _vecs(rng, 2, op.Vh)
    y2 = host(SeedCG(cuda(U), dims, 0.14).apply_M(cuda(x)))
    monkeypatch.setenv("SEEDCG_LINK_ROWS", "9")
    y9 = host(SeedCG(cuda(U), dims, 0.14).apply_M(cuda(x)))
    assert relmax(y2, y9) <= 1e-13
    assert relmax(y2, op.apply_M(x)) <= 1e-13


def test_non_unitary_links_keep_full_links():
    """A field that is not special unitary (here random complex matrices) is read in full: the stencil
    still matches the oracle, which takes the links as given."""
    from paper_0901_3512_amd import SeedCG
    print_case("non-unitary links")
    dims = (4, 4, 4, 4)
    rng = np.random.default_rng(12)
    V = int(np.prod(dims))
    U = 0.6 * (rng.standard_normal((4, V, 3, 3)) + 1j * rng.standard_normal((4, V, 3, 3)))
    op = WilsonEO(U, dims, 0.1)
    x = _vecs(rng, 2, op.Vh)
    for prec in ("fp64", "mixed"):
        s = SeedCG(cuda(U), dims, 0.1, prec=prec)
        y = host(s.apply_M(cuda(x)))
        assert relmax(y, op.apply_M(x)) <= 1e-13, prec
