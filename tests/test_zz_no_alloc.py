"""seedcg_project_noalloc: the contraction P = V^dag R of Algorithm 1 (seeding and reorthogonalisation) with its
split-K partials in the library's static device array, against seedcg_project (which allocates
its partials) on the same inputs.

Bar: bit-identical where seedcg_project's K-chunking fits the static array (same kernels, same
summation order); otherwise normwise relative difference <= 1e-13 (summation order only), and
both within 1e-13 of the plain definition.  Two calls in a row, the second with a smaller input,
so the second reads partials only its own kernels wrote.
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
    U = np.tile(np.eye(3, dtype=np.complex128), (4, 16, 1, 1))
    return SeedCG(cuda(U), (2, 2, 2, 2), 0.1)


# (nv, nr, n) of the first call, then of the second (smaller) call
CASES = [((32, 4, 786432), (5, 3, 1000)),             # 16^3 x 32 vectors, chunking that fits: same bits
         ((32, 11, 786432), (32, 11, 393216)),         # a seeding block at 16^3 x 32: longer K-chunks
         ((300, 2, 200000), (40, 2, 70001)),           # reorthogonalisation coefficients, ragged n
         ((2000, 24, 30000), (700, 24, 12345)),        # partials far beyond seedcg_project's chunking
         ((17, 24, 4097), (1, 1, 1))]


def _kchunk(n, target):
    """seedcg_project's K-chunk: ceil(n / target) rounded up to 32, clamped to [512, 65536]."""
    kc = -(-n // target)
    kc = -(-kc // 32) * 32
    return max(min(kc, 65536), 512)


@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_matches_project_twice(handle, first, second):
    for k, (nv, nr, n) in enumerate((first, second)):
        print_case("project_noalloc", k, nv, nr, n)
        rng = np.random.default_rng(nv * 1009 + nr * 13 + n)
        Vv = cuda(_rand(rng, nv, n))
        R = cuda(_rand(rng, nr, n))
        ref = host(handle.project(Vv, R))
        got = host(handle.project_noalloc(Vv, R))
        kc = _kchunk(n, max(1, 1024 // ((nv + 31) // 32)))
        fits = -(-n // kc) * 2 * nv * nr <= (1 << 19)
        if fits:
            assert np.array_equal(got, ref), (nv, nr, n)
        else:
            assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
        if n * nv <= 2_000_000:
            Vh, Rh = host(Vv), host(R)
            exact = Vh.conj() @ Rh.T
            assert np.linalg.norm(got - exact) <= 1e-13 * np.linalg.norm(exact) * max(1.0, np.log2(n))


def test_noalloc_rejects_sizes_beyond_the_static_array(handle):
    from paper_0901_3512_amd import SeedCGError
    rng = np.random.default_rng(1)
    R = cuda(_rand(rng, 24, 8))
    Vv = cuda(_rand(rng, 10923, 8))     # 10923 * 24 > 262144
    with pytest.raises(SeedCGError) as e:
        handle.project_noalloc(Vv, R)
    assert e.value.code == -1
    with pytest.raises(SeedCGError):
        handle.project_noalloc(cuda(_rand(rng, 2, 8)), cuda(_rand(rng, 25, 8)))
    # the array is still usable after the refusals
    Vv, R = cuda(_rand(rng, 3, 100)), cuda(_rand(rng, 2, 100))
    assert np.array_equal(host(handle.project_noalloc(Vv, R)), host(handle.project(Vv, R)))
