"""The CG step fused into the last stencil launch of q = M p, against the separate update kernel.

In the fused form, the second launch of M p = A^dag A p reduces |A p|^2 = p^dag M p. alpha = rr / p^dag M p
is set before the third launch. The fourth launch applies x += alpha p and r -= alpha q without
storing q. SEEDCG_FUSE_CG=0 selects the separate update kernel.

Bars, for every multi-vector launch shape that carries the fused epilogue (tps 8 and 9 with 1, 2
or 4 vectors per workgroup, tps 10), in FP64 and mixed precision, on 4^4, a ragged 6x4x2x6 and 8^4:
  * every right-hand side reaches the FP64 true relative residual <= 1e-10 by the oracle's M;
  * the CG iteration counts equal the unfused run's to within 1;
  * the solutions agree with the unfused run's to 1e-8 (two 1e-10-residual solutions of one system).
"""
import numpy as np
import pytest

from gpu_helpers import cuda, host, print_case
from oracle.wilson import WilsonEO, flat
from synth.links import random_su3_links

pytestmark = pytest.mark.gpu

SHAPES = [("8", "1"), ("8", "2"), ("8", "4"), ("9", "1"), ("9", "2"), ("9", "4"), ("10", "1"), ("11", "1"), ("11", "2"), ("12", "1")]


def _problem(dims, nrhs=6, seed=11):
    rng = np.random.default_rng(seed)
    U = random_su3_links(dims, 0.4, rng)
    kappa = 0.12
    op = WilsonEO(U, dims, kappa)
    B = rng.standard_normal((nrhs, op.Vh, 4, 3)) + 1j * rng.standard_normal((nrhs, op.Vh, 4, 3))
    return U, kappa, op, B


def _solve(U, dims, kappa, B, prec, fused, shape, monkeypatch):
    from paper_0901_3512_amd import SeedCG
    pre = "SEEDCG_TPS_LO" if prec == "mixed" else "SEEDCG_TPS"
    monkeypatch.setenv(pre, shape[0])
    monkeypatch.setenv(pre.replace("TPS", "VB"), shape[1])
    monkeypatch.setenv("SEEDCG_FUSE_CG", "1" if fused else "0")
    s = SeedCG(cuda(U), dims, kappa, prec=prec, reorth_k=10)
    X, _ = s.solve_seed(cuda(B))
    X, rep = s.solve_rest(cuda(B), X)
    return host(X), rep


# the link-resident stencil (11) runs in FP32 only
PREC_SHAPE = [(p, sh) for p in ("fp64", "mixed") for sh in SHAPES if p == "mixed" or sh[0] != "11"]


@pytest.mark.parametrize("prec,shape", PREC_SHAPE)
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 6), (8, 8, 8, 8)])
def test_fused_cg_step_matches_separate_update(prec, dims, shape, monkeypatch):
    print_case("fused cg", prec, dims, shape)
    U, kappa, op, B = _problem(dims)
    Xf, rf = _solve(U, dims, kappa, B, prec, True, shape, monkeypatch)
    Xu, ru = _solve(U, dims, kappa, B, prec, False, shape, monkeypatch)
    res = np.linalg.norm(flat(B - op.apply_M(Xf)), axis=1) / np.linalg.norm(flat(B), axis=1)
    assert np.all(res <= 1e-10), res
    assert all(abs(a - b) <= 1 for a, b in zip(rf["iters"], ru["iters"])), (rf["iters"], ru["iters"])
    err = np.linalg.norm(flat(Xf - Xu), axis=1) / np.linalg.norm(flat(Xu), axis=1)
    assert np.all(err <= 1e-8), err
    print("fused", rf["iters"], "separate", ru["iters"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fused_cg_step_in_a_batch(prec, monkeypatch):
    """A batch of four configurations in two shape classes (the configuration is one more grid
    dimension of every launch): the fused step matches the separate update kernel, and every
    solution meets the oracle's M."""
    from paper_0901_3512_amd import SeedCGBatch
    print_case("fused cg batch", prec)
    dims = [(4, 4, 4, 4), (6, 4, 2, 6), (4, 4, 4, 4), (6, 4, 2, 6)]
    probs = [_problem(d, nrhs=4, seed=30 + c) for c, d in enumerate(dims)]
    out = {}
    for fused in (True, False):
        monkeypatch.setenv("SEEDCG_FUSE_CG", "1" if fused else "0")
        b = SeedCGBatch([cuda(p[0]) for p in probs], dims, [p[1] for p in probs], 4, prec=prec, reorth_k=10)
        X, reps = b.solve([cuda(p[3]) for p in probs])
        out[fused] = ([host(x) for x in X], [r["iters"] for r in reps])
    for c, (U, kappa, op, B) in enumerate(probs):
        Xf, Xu = out[True][0][c], out[False][0][c]
        res = np.linalg.norm(flat(B - op.apply_M(Xf)), axis=1) / np.linalg.norm(flat(B), axis=1)
        assert np.all(res <= 1e-10), (c, res)
        assert all(abs(a - b) <= 1 for a, b in zip(out[True][1][c], out[False][1][c])), (out[True][1][c], out[False][1][c])
        err = np.linalg.norm(flat(Xf - Xu), axis=1) / np.linalg.norm(flat(Xu), axis=1)
        assert np.all(err <= 1e-8), (c, err)
