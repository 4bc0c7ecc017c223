"""The directions of the paper's own measurements (section 3), on the oracle.

On the 4^4 flux background (near-zero modes apart from the bulk, where seeding pays), with the
first right-hand side seeding the second:
  * Figure 1: the further the first system runs past convergence (m = ceil(past * i_conv)), the
    fewer CG iterations the seeded second system needs;
  * Figure 2: without reorthogonalisation the seeded second system gains less than with it;
  * Table 1: the reorthogonalisation work of the first system (Gram-Schmidt passes, each over
    the i stored vectors) rises as the frequency k falls, and vanishes without it.
These are directions, not the paper's numbers: its configuration and figures are not available.
"""
import pytest

from oracle import seedcg as sc
from test_oracle_seedcg import _flux_case


_cache = {}


@pytest.fixture(scope="module")
def flux2():
    mv, B = _flux_case((1, 1))
    return mv, B[:2]


def _rhs2_iters(mv, B, k, past):
    """Algorithm 1 on RHS 1 seeding RHS 2, then CG on RHS 2 from its seeded guess (cached per k, past)."""
    if (k, past) not in _cache:
        out = sc.seed_cg(mv, B, k=k, tol=1e-10, past=past)
        _, it, r, _ = sc.cg(mv, B[1], out["X"][1], tol=1e-10)
        assert r <= 1e-10
        _cache[(k, past)] = (out, it)
    return _cache[(k, past)]


def test_fig1_running_past_convergence_helps_the_seeded_system(flux2):
    mv, B = flux2
    its = [_rhs2_iters(mv, B, 10, p)[1] for p in (1.0, 1.2, 1.5, 2.0)]
    assert all(a >= b for a, b in zip(its, its[1:])), its
    assert its[-1] < its[0], its


def test_fig2_no_reorthogonalisation_gains_less(flux2):
    mv, B = flux2
    _, cold, _, _ = sc.cg(mv, B[1], None, tol=1e-10)
    _, it_none = _rhs2_iters(mv, B, 0, 1.5)
    _, it_k10 = _rhs2_iters(mv, B, 10, 1.5)
    _, it_k20 = _rhs2_iters(mv, B, 20, 1.5)
    assert it_k10 < it_none and it_k20 < it_none, (it_none, it_k10, it_k20)
    assert max(it_k10, it_k20) < 0.5 * cold


def test_table1_reorthogonalisation_work_rises_as_k_falls(flux2):
    mv, B = flux2
    work = []
    for k in (0, 20, 10, 5):
        out, _ = _rhs2_iters(mv, B, k, 1.5)
        # each pass at step i reads the i - 1 (or i) stored vectors: count them
        steps = range(k, out["m"] + 1, k) if k else []
        work.append((out["reorth_passes"], sum(steps)))
    passes = [w[0] for w in work]
    assert passes[0] == 0 and passes[1] < passes[2] < passes[3], passes
    vecs = [w[1] for w in work]
    assert vecs[0] == 0 and vecs[1] < vecs[2] < vecs[3], vecs
