"""Kernels (b) and (c): P = V^dag R on the matrix cores and X += W E, against their definitions.

The oracle of a contraction is its plain definition (a numpy product in FP64).
FP64 bar: normwise relative error <= 1e-13 (split-K summation order only).
"""
import numpy as np
import pytest

from gpu_helpers import cuda, host, print_case

pytestmark = pytest.mark.gpu


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.fixture(scope="module")
def handle():
    from paper_0901_3512_amd import SeedCG
    dims = (2, 2, 2, 2)
    U = np.tile(np.eye(3, dtype=np.complex128), (4, 16, 1, 1))
    return SeedCG(cuda(U), dims, 0.1)


@pytest.mark.parametrize("nv,nr,n", [(1, 1, 1), (5, 3, 100), (32, 11, 1536), (32, 23, 4097), (70, 2, 20000),
                                     (16, 8, 33), (3, 24, 70001), (33, 1, 5000)])
def test_project_matches_definition(handle, nv, nr, n):
    print_case("project", nv, nr, n)
    rng = np.random.default_rng(nv * 1000 + nr)
    Vv = _rand(rng, nv, n)
    R = _rand(rng, nr, n)
    P = host(handle.project(cuda(Vv), cuda(R)))
    ref = Vv.conj() @ R.T
    assert np.linalg.norm(P - ref) <= 1e-13 * np.linalg.norm(ref) * max(1.0, np.log2(n))


@pytest.mark.parametrize("nw,nx,n", [(1, 1, 1), (4, 3, 1000), (32, 11, 12289), (20, 23, 777), (32, 48, 300)])
def test_update_matches_definition(handle, nw, nx, n):
    print_case("update", nw, nx, n)
    rng = np.random.default_rng(nw + 7 * nx)
    W = _rand(rng, nw, n)
    E = _rand(rng, nw, nx)
    X = _rand(rng, nx, n)
    ref = X + (W.T @ E).T
    out = host(handle.update(cuda(W), cuda(E), cuda(X.copy())))
    assert np.linalg.norm(out - ref) <= 1e-14 * np.linalg.norm(ref) * nw


def test_project_rejects_too_many_columns(handle):
    from paper_0901_3512_amd import SeedCGError
    rng = np.random.default_rng(0)
    with pytest.raises(SeedCGError):
        handle.project(cuda(_rand(rng, 2, 10)), cuda(_rand(rng, 25, 10)))
