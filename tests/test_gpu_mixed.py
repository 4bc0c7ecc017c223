"""Mixed precision (FP32 stencil, basis and CG; optional BF16 links; FP64 reliable updates).

  * The inner operator against the oracle applied to the same rounded inputs (links rounded
    to FP32 or to BF16 by round-to-nearest-even, x rounded to FP32): this isolates the FP32
    arithmetic, bar 5e-6 relative to max |M x|.
  * Full solves: every right-hand side reaches an FP64 true relative residual <= 1e-10 by the
    oracle's FP64 M, and agrees with the dense FP64 solution to 1e-8.
"""
import numpy as np
import pytest

from gpu_helpers import cuda, host, print_case, relmax
from oracle import seedcg as osc
from oracle.wilson import WilsonEO, dense, flat, matvec_M
from synth.configs import make_inputs
from synth.links import random_su3_links

pytestmark = pytest.mark.gpu


def round_fp32(a):
    return a.real.astype(np.float32).astype(np.float64) + 1j * a.imag.astype(np.float32).astype(np.float64)


def _bf16(x):
    f = np.ascontiguousarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return b.view(np.float32).astype(np.float64)


def round_bf16(a):
    return _bf16(a.real) + 1j * _bf16(a.imag)


@pytest.mark.parametrize("prec,rounder", [("mixed", round_fp32), ("mixed_bf16", round_bf16), ("mixed_cg", round_fp32)])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 6), (8, 8, 8, 16), (32, 34, 2, 2)])
@pytest.mark.parametrize("shape", [("3", "1"), ("6", "1"), ("7", "2"), ("7", "4"), ("8", "1"), ("8", "2"), ("8", "4"),
                                   ("9", "1"), ("9", "2"), ("9", "4"), ("10", "1"), ("11", "1"), ("11", "2"), ("12", "1")])
def test_inner_operator_matches_oracle_on_rounded_inputs(prec, rounder, dims, shape, monkeypatch):
    from paper_0901_3512_amd import SeedCG
    print_case("inner", prec, dims, shape)
    monkeypatch.setenv("SEEDCG_TPS_LO", shape[0])
    monkeypatch.setenv("SEEDCG_VB_LO", shape[1])
    rng = np.random.default_rng(4)
    U = random_su3_links(dims, 0.4, rng)
    kappa = 0.13
    op = WilsonEO(rounder(U), dims, kappa)
    Vh = op.Vh
    x = round_fp32(rng.standard_normal((5, Vh, 4, 3)) + 1j * rng.standard_normal((5, Vh, 4, 3)))
    s = SeedCG(cuda(U), dims, kappa, prec=prec)
    y = host(s.apply_M_inner(cuda(x)))
    assert relmax(y, op.apply_M(x)) <= 5e-6


@pytest.fixture(scope="module")
def t8():
    """8^4, kappa 0.13 (physical branch): the FP32 operator keeps Lanczos well defined."""
    U, phi, kappa = make_inputs("t8")
    dims = (8, 8, 8, 8)
    op = WilsonEO(U, dims, kappa)
    B = op.apply_Adag(phi)
    mv = matvec_M(op)
    ref = osc.seed_cg(mv, flat(B), k=10, tol=1e-10, past=1.5)
    xs = np.stack([osc.cg(mv, flat(B)[j], ref["X"][j], tol=1e-13)[0] for j in range(B.shape[0])])
    return dict(U=U, dims=dims, kappa=kappa, B=B, mv=mv, xs=xs, ref=ref)


@pytest.fixture(scope="module")
def c1():
    U, phi, kappa = make_inputs("c1")
    dims = (4, 4, 4, 4)
    op = WilsonEO(U, dims, kappa)
    B = op.apply_Adag(phi)
    mv = matvec_M(op)
    xs = np.linalg.solve(dense(mv, 12 * op.Vh), flat(B).T).T
    return dict(U=U, dims=dims, kappa=kappa, B=B, mv=mv, xs=xs)


@pytest.mark.parametrize("prec", ["mixed", "mixed_bf16"])
def test_mixed_solve_reaches_fp64_tolerance(t8, prec):
    from paper_0901_3512_amd import SeedCG
    print_case("mixed solve", prec)
    s = SeedCG(cuda(t8["U"]), t8["dims"], t8["kappa"], prec=prec, reorth_k=10, reliable_every=50, max_iter=5000)
    Bd = cuda(t8["B"])
    X, rs = s.solve_seed(Bd)
    assert rs["seed_status"] == "ok"
    res_seed = osc.true_relres(t8["mv"], flat(t8["B"]), flat(host(X)))
    assert np.all(res_seed < 1.0)
    X, rr = s.solve_rest(Bd, X)
    x = flat(host(X))
    res = osc.true_relres(t8["mv"], flat(t8["B"]), x)
    assert np.all(res <= 1e-10), res
    err = np.linalg.norm(x - t8["xs"], axis=1) / np.linalg.norm(t8["xs"], axis=1)
    assert np.all(err <= 1e-8), err


def test_mixed_seed_basis_orthogonality_and_tridiag(t8):
    """FP32 basis with FP64 reorthogonalisation coefficients stays orthogonal to FP32 accuracy, and
    its T matches the FP64 oracle's in the first steps to FP32 accuracy."""
    from paper_0901_3512_amd import SeedCG
    print_case("mixed basis")
    s = SeedCG(cuda(t8["U"]), t8["dims"], t8["kappa"], prec="mixed", reorth_k=10)
    X, rs = s.solve_seed(cuda(t8["B"]))
    m = rs["m"]
    assert abs(m - t8["ref"]["m"]) <= max(2, m // 20)
    Vg = np.stack([flat(host(s.get_basis_vector(i))) for i in range(1, m + 1)])
    assert osc.orth_loss(Vg) <= 1e-5
    a, b = s.get_tridiag()
    n = 10
    ref = t8["ref"]
    assert np.max(np.abs(np.array(a[:n]) - ref["alpha"][:n]) / np.abs(ref["alpha"][:n])) <= 1e-5


def test_mixed_at_large_kappa_still_converges(c1):
    """At kappa = 0.8 the hopping term is ~40x the identity and FP32 rounding breaks the Lanczos
    invariants (the same happens to the oracle's Algorithm 1 run on an FP32-rounded M); the seed
    reports it and plain CG with FP64 reliable updates still reaches the FP64 tolerance."""
    from paper_0901_3512_amd import SeedCG
    print_case("mixed large kappa")
    s = SeedCG(cuda(c1["U"]), c1["dims"], c1["kappa"], prec="mixed", reorth_k=10, max_iter=20000)
    Bd = cuda(c1["B"])
    X, rs = s.solve_seed(Bd)
    X, rr = s.solve_rest(Bd, X)
    x = flat(host(X))
    res = osc.true_relres(c1["mv"], flat(c1["B"]), x)
    assert np.all(res <= 1e-10), res
    err = np.linalg.norm(x - c1["xs"], axis=1) / np.linalg.norm(c1["xs"], axis=1)
    assert np.all(err <= 1e-8), err


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 6), (8, 8, 8, 8)])
def test_mixed_cg_iterations_track_fp64(dims):
    """Regression of the reliable updates when CG converges fast (a rough random field, kappa 0.12):
    the decade trigger works from the first iteration on, and a true residual far above the
    recursive one restarts the direction. Mixed CG then needs at most 1.5x FP64's iterations + 10
    per right-hand side. Before the fix, two of five systems crawled for over 1000 iterations at a
    frozen true residual of 3e-6."""
    from paper_0901_3512_amd import SeedCG
    print_case("mixed iterations vs fp64", dims)
    rng = np.random.default_rng(11)
    U = random_su3_links(dims, 0.4, rng)
    op = WilsonEO(U, dims, 0.12)
    B = rng.standard_normal((6, op.Vh, 4, 3)) + 1j * rng.standard_normal((6, op.Vh, 4, 3))
    its = {}
    for prec in ("fp64", "mixed"):
        s = SeedCG(cuda(U), dims, 0.12, prec=prec, reorth_k=10)
        X, _ = s.solve_seed(cuda(B))
        X, rep = s.solve_rest(cuda(B), X)
        res = np.linalg.norm(flat(B - op.apply_M(host(X))), axis=1) / np.linalg.norm(flat(B), axis=1)
        assert np.all(res <= 1e-10), (prec, res)
        its[prec] = rep["iters"]
    assert all(m <= 1.5 * f + 10 for m, f in zip(its["mixed"][1:], its["fp64"][1:])), its
    print("iterations", its)


def test_mixed_cg_mode_keeps_the_seeding_gain():
    """MIXED_FP32_CG (FP64 Lanczos, basis and seeding; FP32 CG with FP64 reliable updates) on the
    4^4 flux background at kappa 0.17, whose near-zero modes stand apart from the bulk: every
    solution within 1e-8 of the dense solve; the seed run identical to the FP64 one (same m, bit
    for bit the same seeded guesses); the seeded systems within 1.5x + 10 of FP64's CG iterations.
    The FP32 basis of MIXED_FP32 is reported beside it. The mode with deflation (FP32 Ritz vectors)
    also solves within 1e-8; training K needs a seed solve first."""
    from dataclasses import replace

    from paper_0901_3512_amd import SeedCG, SeedCGError
    from synth.configs import CONFIGS, make_links, make_sources
    print_case("mixed_cg flux 4^4")
    cfg = replace(CONFIGS["c1"], flux=(1, 1))
    U = make_links(cfg)
    op = WilsonEO(U, cfg.dims, 0.17)
    mv = matvec_M(op)
    B = op.apply_Adag(make_sources(cfg))
    xs = np.linalg.solve(dense(mv, 12 * op.Vh), flat(B).T).T
    out = {}
    for prec in ("fp64", "mixed_cg", "mixed"):
        s = SeedCG(cuda(U), cfg.dims, 0.17, prec=prec, reorth_k=10)
        X0, rs = s.solve_seed(cuda(B))
        X, rr = s.solve_rest(cuda(B), X0.clone())
        err = np.linalg.norm(flat(host(X)) - xs, axis=1) / np.linalg.norm(xs, axis=1)
        assert np.all(err <= 1e-8), (prec, err)
        out[prec] = (rs["m"], host(X0), rr["iters"])
    assert out["mixed_cg"][0] == out["fp64"][0]
    assert np.array_equal(out["mixed_cg"][1], out["fp64"][1])
    assert all(m <= 1.5 * f + 10 for m, f in zip(out["mixed_cg"][2][1:], out["fp64"][2][1:])), out
    print("seeded CG iterations: fp64", out["fp64"][2], "mixed_cg", out["mixed_cg"][2], "mixed", out["mixed"][2])
    # deflated FP32 CG from the FP64 Algorithm 1 (the Ritz vectors and M W in FP32)
    sd = SeedCG(cuda(U), cfg.dims, 0.17, prec="mixed_cg", reorth_k=10, deflate=4)
    X0, _ = sd.solve_seed(cuda(B))
    X, rd = sd.solve_rest(cuda(B), X0.clone())
    err = np.linalg.norm(flat(host(X)) - xs, axis=1) / np.linalg.norm(xs, axis=1)
    assert np.all(err <= 1e-8), ("mixed_cg deflated", err)
    s = SeedCG(cuda(U), cfg.dims, 0.17, prec="mixed_cg")
    with pytest.raises(SeedCGError):
        s.train_precond(steps=1)   # no seed solve yet
    # the other solvers of the handle: repeated seeding (FP64 Lanczos per system, FP32 CG). Its
    # stop is the 1e-10 residual, and here cond(M) = 2.3e4, so the forward error may reach
    # cond x 1e-10 = 2.3e-6 (3.9e-8 measured for one system).
    X, rr = s.solve_repeated(cuda(B))
    res = np.linalg.norm(flat(B - op.apply_M(host(X))), axis=1) / np.linalg.norm(flat(B), axis=1)
    assert np.all(res <= 1e-10), res
    err = np.linalg.norm(flat(host(X)) - xs, axis=1) / np.linalg.norm(xs, axis=1)
    assert np.all(err <= 2.3e4 * 1e-10), err


@pytest.mark.parametrize("prec", ["fp64", "mixed_cg"])
def test_fp32_basis_copy_of_fp64_lanczos(t8, prec):
    """basis_fp32: the FP64 Lanczos recurrence with each finished v_i rounded into an FP32 basis, the
    projections contracting that basis on the FP64 matrix cores (8^4, k = 10).  Against the oracle:
    m and i_conv within one step, the first 20 Lanczos coefficients to 1e-8 relative (the FP32 copy
    enters T only through the reorthogonalisation coefficients, whose rounding errors are incoherent
    with the basis), the seeded guesses to 1e-6; the stored vectors are the FP32 roundings of an
    orthonormal set (|V^dag V - 1| <= 1e-6); every solution within 1e-8 of the FP64 solution and at
    an FP64 true residual <= 1e-10."""
    from paper_0901_3512_amd import SeedCG
    print_case("fp32 basis copy", prec)
    ref = t8["ref"]
    s = SeedCG(cuda(t8["U"]), t8["dims"], t8["kappa"], prec=prec, reorth_k=10, basis_fp32=True)
    X, rs = s.solve_seed(cuda(t8["B"]))
    assert abs(rs["m"] - ref["m"]) <= 1 and abs(rs["i_conv"] - ref["i_conv"]) <= 1, (rs["m"], ref["m"])
    a, b = s.get_tridiag()
    n = min(20, len(a))
    assert np.max(np.abs(np.array(a[:n]) - ref["alpha"][:n]) / np.abs(ref["alpha"][:n])) <= 1e-8
    assert np.max(np.abs(np.array(b[:n]) - ref["beta"][:n]) / ref["beta"][:n]) <= 1e-8
    rel = np.linalg.norm(flat(host(X)) - ref["X"], axis=1) / np.linalg.norm(ref["X"], axis=1)
    assert np.max(rel[1:]) <= 1e-6, rel
    V = np.stack([flat(host(s.get_basis_vector(i))) for i in range(1, rs["m"] + 1)])
    assert np.all(V == V.astype(np.complex64).astype(np.complex128))   # FP32-representable entries
    assert osc.orth_loss(V) <= 1e-6
    X, rr = s.solve_rest(cuda(t8["B"]), X)
    assert np.all(osc.true_relres(t8["mv"], flat(t8["B"]), flat(host(X))) <= 1e-10)
    err = np.linalg.norm(flat(host(X)) - t8["xs"], axis=1) / np.linalg.norm(t8["xs"], axis=1)
    assert np.max(err) <= 1e-8, err
    print("fp32 basis copy", prec, "m", rs["m"], "iters", rr["iters"])


@pytest.mark.parametrize("prec", ["fp64", "mixed_cg"])
def test_fp32_reorth_copy_of_fp64_basis(t8, prec):
    """basis_fp32 = "reorth": the FP64 basis serves the seeding, and an FP32 copy of every finished v_i
    serves the periodic reorthogonalisation only (8^4, k = 10).  Against the oracle: m and i_conv within
    one step, the first 20 Lanczos coefficients to 1e-8 relative (the copy enters T only through the
    reorthogonalisation coefficients), the seeded guesses to 1e-6; the basis vectors handed out are the
    FP64 ones (not FP32-representable) and orthonormal to FP32 rounding; every solution within 1e-8 of
    the FP64 solution and at an FP64 true residual <= 1e-10."""
    from paper_0901_3512_amd import SeedCG
    print_case("fp32 reorth copy", prec)
    ref = t8["ref"]
    s = SeedCG(cuda(t8["U"]), t8["dims"], t8["kappa"], prec=prec, reorth_k=10, basis_fp32="reorth")
    X, rs = s.solve_seed(cuda(t8["B"]))
    assert abs(rs["m"] - ref["m"]) <= 1 and abs(rs["i_conv"] - ref["i_conv"]) <= 1, (rs["m"], ref["m"])
    a, b = s.get_tridiag()
    n = min(20, len(a))
    assert np.max(np.abs(np.array(a[:n]) - ref["alpha"][:n]) / np.abs(ref["alpha"][:n])) <= 1e-8
    assert np.max(np.abs(np.array(b[:n]) - ref["beta"][:n]) / ref["beta"][:n]) <= 1e-8
    rel = np.linalg.norm(flat(host(X)) - ref["X"], axis=1) / np.linalg.norm(ref["X"], axis=1)
    assert np.max(rel[1:]) <= 1e-6, rel
    V = np.stack([flat(host(s.get_basis_vector(i))) for i in range(1, rs["m"] + 1)])
    assert not np.all(V == V.astype(np.complex64).astype(np.complex128))   # the FP64 vectors
    assert osc.orth_loss(V) <= 1e-6
    X, rr = s.solve_rest(cuda(t8["B"]), X)
    assert np.all(osc.true_relres(t8["mv"], flat(t8["B"]), flat(host(X))) <= 1e-10)
    err = np.linalg.norm(flat(host(X)) - t8["xs"], axis=1) / np.linalg.norm(t8["xs"], axis=1)
    assert np.max(err) <= 1e-8, err
    print("fp32 reorth copy", prec, "m", rs["m"], "orth", osc.orth_loss(V), "iters", rr["iters"])


def test_reorth_copy_keeps_the_seeding_gain_that_an_fp32_basis_loses():
    """On 8^4 with one flux quantum through two planes (kappa 0.14: near-zero modes apart from the
    bulk, where the seeded guesses carry most of the solution), FP64 Lanczos with FP32 CG, six point
    sources: the FP32 reorthogonalisation copy of the FP64 basis leaves every seeded system's CG
    iterations within 2 of the FP64 basis' (the oracle, with the basis rounded for the
    reorthogonalisation only, gives the same counts: 58-59), while the FP32 basis, whose seeding
    projections use the rounded vectors, needs at least 15% more on average (oracle: 80-82)."""
    from paper_0901_3512_amd import SeedCG
    from synth.configs import CONFIGS, make_links, with_changes
    from synth.sources import point_sources
    dims = (8, 8, 8, 8)
    U = make_links(with_changes(CONFIGS["c5"], dims=dims, flux=(1, 1)))
    op = WilsonEO(U, dims, 0.14)
    B = op.apply_Adag(point_sources(dims, 6))
    its = {}
    for mode in (False, "reorth", True):
        print_case("seeding gain, basis", mode)
        s = SeedCG(cuda(U), dims, 0.14, prec="mixed_cg", reorth_k=10, basis_fp32=mode)
        X, _ = s.solve_seed(cuda(B))
        X, rr = s.solve_rest(cuda(B), X)
        assert np.all(osc.true_relres(matvec_M(op), flat(B), flat(host(X))) <= 1e-10)
        its[mode] = np.array(rr["iters"][1:])
        s.close()
    print("seeded CG iterations", {str(k): v.tolist() for k, v in its.items()})
    assert np.max(np.abs(its["reorth"] - its[False])) <= 2, its
    assert its[True].mean() >= 1.15 * its[False].mean(), its


def test_fp32_basis_copy_refused_for_batches():
    from paper_0901_3512_amd import SeedCGError
    from paper_0901_3512_amd.seedcg import Params, load_library
    import ctypes
    lib = load_library()
    p = Params()
    lib.seedcg_default_params(ctypes.byref(p))
    p.basis_fp32 = 1
    dims = (ctypes.c_int32 * 4)(4, 4, 4, 4)
    kap = (ctypes.c_double * 1)(0.12)
    links = (ctypes.c_void_p * 1)(None)
    h = ctypes.c_void_p()
    rc = lib.seedcg_create_batch(1, dims, kap, links, 3, ctypes.byref(p), ctypes.byref(h))
    assert rc != 0 and not h.value
