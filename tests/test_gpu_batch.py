"""Batches of configurations (seedcg_create_batch / seedcg_solve_batch) on the GPU.

Bars:
  * every right-hand side of every configuration reaches the FP64 true relative residual 1e-10,
    judged by the oracle's M, and (FP64) agrees with the oracle's dense solve to 1e-8;
  * with fixed launch shapes, every configuration of a batch gets bit for bit the solution, m and
    iteration counts that a handle of its own gets (a batch launch runs the same kernels with the
    configuration as one more grid dimension);
  * CG iterations replayed from hipGraphs give bit for bit the results of eager launches;
  * the edge cases: a class of one configuration, a zero right-hand side, nrhs = 1.
"""
import os

import numpy as np
import pytest

from gpu_helpers import cuda, host, print_case
from oracle import seedcg as osc
from oracle.wilson import WilsonEO, dense, flat, matvec_M
from synth.links import random_su3_links

pytestmark = pytest.mark.gpu

# three shapes: a class of three, a class of two, a class of one
SHAPES = [(4, 4, 4, 4), (4, 2, 4, 6), (4, 4, 4, 4), (6, 4, 4, 4), (4, 2, 4, 6), (4, 4, 4, 4)]
KAPPAS = [0.12, 0.125, 0.13, 0.12, 0.118, 0.135]
NRHS = 4


def _config(c, nrhs=NRHS, zero_rhs=None):
    dims = SHAPES[c]
    rng = np.random.default_rng([0xBA7C4, c])
    U = random_su3_links(dims, 0.4, rng)
    op = WilsonEO(U, dims, KAPPAS[c])
    phi = rng.standard_normal((nrhs, op.Vh, 4, 3)) + 1j * rng.standard_normal((nrhs, op.Vh, 4, 3))
    B = op.apply_Adag(phi)
    if zero_rhs is not None:
        B[zero_rhs] = 0.0
    return dict(dims=dims, U=U, kappa=KAPPAS[c], op=op, B=B, mv=matvec_M(op))


@pytest.fixture(scope="module")
def cfgs():
    return [_config(c) for c in range(len(SHAPES))]


def _batch(cfgs, prec, **kw):
    from paper_0901_3512_amd import SeedCGBatch
    return SeedCGBatch([cuda(c["U"]) for c in cfgs], [c["dims"] for c in cfgs], [c["kappa"] for c in cfgs],
                       cfgs[0]["B"].shape[0], prec=prec, reorth_k=10, **kw)


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_cg"])
def test_batch_matches_oracle(cfgs, prec):
    print_case("batch oracle", prec)
    b = _batch(cfgs, prec, m_max=400)
    info = b.info()
    assert info["nclass"] == 3 and info["class_of"] == [0, 1, 0, 2, 1, 0] and info["m_cap"] == [400] * 3
    X, reps = b.solve([cuda(c["B"]) for c in cfgs])
    for c, (cfg, x, rep) in enumerate(zip(cfgs, X, reps)):
        xb = flat(host(x))
        res = osc.true_relres(cfg["mv"], flat(cfg["B"]), xb)
        assert np.all(res <= 1e-10), (c, res)
        assert np.allclose(rep["true_relres"], res, rtol=1e-3, atol=1e-14)
        if prec != "mixed":   # FP64 Algorithm 1 (with an FP32 CG in mixed_cg)
            Md = dense(cfg["mv"], 12 * cfg["op"].Vh)
            xs = np.linalg.solve(Md, flat(cfg["B"]).T).T
            err = np.linalg.norm(xb - xs, axis=1) / np.linalg.norm(xs, axis=1)
            assert np.all(err <= 1e-8), (c, err)
            ref = osc.seed_cg(cfg["mv"], flat(cfg["B"]), k=10, tol=1e-10, past=1.5)
            assert abs(rep["m"] - ref["m"]) <= 1 and abs(rep["i_conv"] - ref["i_conv"]) <= 1, (c, rep["m"], ref["m"])
        print("batch", prec, c, cfg["dims"], "m", rep["m"], "iters", rep["iters"])


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_cg"])
@pytest.mark.parametrize("shape", [None, ("9", "2"), ("10", "1"), ("3", "1"), ("11", "2"), ("12", "1")])
def test_batch_equals_separate_handles(cfgs, prec, shape, monkeypatch):
    """shape: a stencil launch shape (lanes-per-site code, vectors per workgroup) forced on both
    sides; None = the default one."""
    from paper_0901_3512_amd import SeedCG
    print_case("batch vs single", prec, shape)
    if shape:
        for k, v in (("SEEDCG_TPS", shape[0]), ("SEEDCG_TPS_LO", shape[0]), ("SEEDCG_VB", shape[1]), ("SEEDCG_VB_LO", shape[1])):
            monkeypatch.setenv(k, v)
    b = _batch(cfgs, prec, m_max=300, autotune=False)
    Xb, reps = b.solve([cuda(c["B"]) for c in cfgs])
    for c, cfg in enumerate(cfgs):
        s = SeedCG(cuda(cfg["U"]), cfg["dims"], cfg["kappa"], prec=prec, reorth_k=10, m_max=300, autotune=False)
        B = cuda(cfg["B"])
        X, rs = s.solve_seed(B)
        X, rr = s.solve_rest(B, X)
        assert rs["m"] == reps[c]["m"] and rs["i_conv"] == reps[c]["i_conv"]
        assert [rr["iters"][j] + (rs["m"] if j == 0 else 0) for j in range(NRHS)] == reps[c]["iters"]
        assert np.array_equal(host(X), host(Xb[c])), c


def test_graph_replay_equals_eager(cfgs):
    print_case("graphs vs eager")
    outs = []
    for flag in ("1", "0"):
        os.environ["SEEDCG_GRAPHS"] = flag
        try:
            b = _batch(cfgs, "mixed", m_max=300, autotune=False)
        finally:
            os.environ.pop("SEEDCG_GRAPHS", None)
        X, reps = b.solve([cuda(c["B"]) for c in cfgs])
        outs.append(([host(x) for x in X], [r["iters"] for r in reps]))
        b.close()
    # and a second solve on the same graphs: replays after the first
    b = _batch(cfgs, "mixed", m_max=300, autotune=False)
    for _ in range(2):
        X, reps = b.solve([cuda(c["B"]) for c in cfgs])
        assert [r["iters"] for r in reps] == outs[1][1]
        assert all(np.array_equal(host(x), y) for x, y in zip(X, outs[1][0]))
    assert outs[0][1] == outs[1][1]
    assert all(np.array_equal(x, y) for x, y in zip(outs[0][0], outs[1][0]))


def test_batch_edge_cases():
    from paper_0901_3512_amd import SeedCGBatch
    print_case("batch edges")
    # a zero right-hand side in one configuration, and a batch of one configuration
    cfgs = [_config(0, zero_rhs=2), _config(3)]
    b = _batch(cfgs, "fp64", m_max=300)
    X, reps = b.solve([cuda(c["B"]) for c in cfgs])
    assert np.all(host(X[0])[2] == 0) and reps[0]["iters"][2] == 0
    for c, cfg in enumerate(cfgs):
        live = [j for j in range(NRHS) if np.any(cfg["B"][j] != 0)]
        res = osc.true_relres(cfg["mv"], flat(cfg["B"][live]), flat(host(X[c])[live]))
        assert np.all(res <= 1e-10)
    one = _config(1)
    b1 = SeedCGBatch([cuda(one["U"])], [one["dims"]], [one["kappa"]], NRHS, prec="mixed", m_max=300)
    X1, r1 = b1.solve([cuda(one["B"])])
    assert np.all(osc.true_relres(one["mv"], flat(one["B"]), flat(host(X1[0]))) <= 1e-10)
    # nrhs = 1: Algorithm 1 alone, then CG only if the Lanczos iterate missed tol
    c1 = [_config(0, nrhs=1), _config(1, nrhs=1)]
    b2 = _batch(c1, "fp64", m_max=300)
    X2, r2 = b2.solve([cuda(c["B"]) for c in c1])
    for c, cfg in enumerate(c1):
        assert np.all(osc.true_relres(cfg["mv"], flat(cfg["B"]), flat(host(X2[c]))) <= 1e-10)


def test_batch_argument_errors(cfgs):
    from paper_0901_3512_amd import SeedCGBatch, SeedCGError
    print_case("batch errors")
    with pytest.raises(ValueError):
        SeedCGBatch([cuda(cfgs[0]["U"])], [cfgs[0]["dims"], cfgs[1]["dims"]], [0.1], 4)
    with pytest.raises(SeedCGError):
        SeedCGBatch([cuda(cfgs[0]["U"])], [cfgs[0]["dims"]], [0.12], 30)   # nrhs > 25
    b = _batch(cfgs[:2], "fp64", m_max=100)
    with pytest.raises(ValueError):
        b.solve([cuda(cfgs[0]["B"])])


def _member_inputs(name):
    from synth.configs import batch_members, make_links, make_sources
    m = {c.name: c for c in batch_members()}[name]
    return make_links(m), make_sources(m)


def _c4_kappas_ready():
    import json
    from synth import configs
    path = configs._KAPPA_FILE
    if not os.path.exists(path):
        return False
    tab = json.load(open(path))
    return all(m.name in tab for m in configs.batch_members())


@pytest.mark.skipif(not _c4_kappas_ready(), reason="the oracle's kappa search has not covered every batch member")
def test_c4_full_batch_sampled_against_oracle():
    """The batched workload at its full size (64 configurations, 12 point sources each, mixed precision),
    in the launch configuration the benchmark times: every right-hand side reports an FP64 true residual
    <= 1e-10, and for one member of every shape the oracle's M confirms it on all 12 solutions."""
    from paper_0901_3512_amd import SeedCG, SeedCGBatch
    from synth.configs import batch_members, kappa_for
    import torch
    members = batch_members()
    print_case("c4 full batch", len(members))
    inputs = [_member_inputs(m.name) for m in members]   # host only (this process already uses the GPU)
    kappas = [kappa_for(m) for m in members]
    links = [cuda(U) for U, _ in inputs]
    B = []
    for m, k, (U, phi), Ud in zip(members, kappas, inputs, links):
        s = SeedCG(Ud, m.dims, k, autotune=False)
        B.append(s.apply_A(cuda(phi), dagger=True))
        s.close()
    b = SeedCGBatch(links, [m.dims for m in members], kappas, 12, prec=members[0].prec, reorth_k=members[0].reorth_k,
                    tol=members[0].tol)
    X, reps = b.solve(B)
    torch.cuda.synchronize()
    worst = max(max(r["true_relres"]) for r in reps)
    assert worst <= 1e-10, worst
    seen = set()
    for c, m in enumerate(members):
        if m.dims in seen:
            continue
        seen.add(m.dims)
        op = WilsonEO(inputs[c][0], m.dims, kappas[c])
        B_ref = op.apply_Adag(inputs[c][1])      # the oracle's own right-hand sides
        res = osc.true_relres(matvec_M(op), flat(B_ref), flat(host(X[c])))
        assert np.all(res <= 1e-10), (m.name, res)
        print("c4", m.name, m.dims, "m", reps[c]["m"], "iters", reps[c]["iters"], "oracle relres", float(res.max()))


def test_timing_counts_every_stencil_launch(cfgs):
    """get_timing's last two values count every stencil launch of the batch and its algorithmic
    bytes: with every launch sampled they equal the sampled sums; sampling every third launch leaves
    them unchanged (the same solve issues the same launches) and samples fewer."""
    print_case("batch timing totals")
    b = _batch(cfgs, "mixed", m_max=300, autotune=False)
    B = [cuda(c["B"]) for c in cfgs]
    b.set_timing(1, 16384)
    b.solve(B)
    all1 = b.get_timing()
    b.set_timing(3, 16384)
    b.solve(B)
    all3 = b.get_timing()
    b.set_timing(0, 0)
    b.close()
    assert all1["seen"] > 0
    assert all1["launches"] == all1["seen"]
    assert all1["seen_bytes"] == pytest.approx(all1["bytes"], rel=1e-12)
    assert all3["seen"] == all1["seen"] and all3["seen_bytes"] == pytest.approx(all1["seen_bytes"], rel=1e-12)
    assert 0 < all3["launches"] < all3["seen"] and 0 < all3["bytes"] < all3["seen_bytes"]
