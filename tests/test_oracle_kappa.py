"""Pins of the oracle's kappa search (it sets every workload's hopping parameter).

The search reads lambda_min / lambda_max of M = A^dag A (section 3) either from a dense eigvalsh or
from a plain Lanczos run stopped when the lowest Ritz pair's residual bound is below 2% of the Ritz
value.  Pinned here against dense eigenvalues, which do not share its code:
  * the Lanczos extremes: lambda_min <= theta_min <= 1.02 lambda_min (Cauchy interlacing and the 2%
    stop rule) and 0.99 lambda_max <= theta_max <= lambda_max, on 4^4 and 4^3 x 8 operators;
  * the scan and bisection: on the 4^4 correctness workload the search reproduces the stored kappa
    and every stored evaluation, and the dense ratio at that kappa meets the target to 0.05 in log10;
  * the same with Lanczos extremes forced, on a 4^4 flux background whose near-zero modes make the
    target reachable near the critical kappa: the dense ratio at the kappa found meets the target;
  * the dip branch: when the ratio turns upward before reaching the target, the search returns the
    minimum of a dense kappa grid around it (and records the target as unreachable).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle.kappa_search import OUT, extremes_dense, extremes_lanczos, search
from oracle.wilson import WilsonEO
from synth.configs import CONFIGS, make_links, with_changes
from synth.links import flux_background


def _quiet(*a, **k):
    pass


@pytest.fixture(scope="module")
def c1_links():
    return make_links(CONFIGS["c1"])


@pytest.mark.parametrize("dims,kappa", [((4, 4, 4, 4), 0.12), ((4, 4, 4, 4), 0.15), ((4, 4, 4, 4), 0.5),
                                        ((4, 4, 4, 8), 0.14), ((4, 4, 4, 8), 0.16)])
def test_lanczos_extremes_within_the_stop_rule(dims, kappa):
    U = make_links(with_changes(CONFIGS["c1"], dims=dims))
    op = WilsonEO(U, dims, kappa)
    lo, hi, _ = extremes_dense(op)
    tlo, thi, how = extremes_lanczos(op)
    assert how.startswith("lanczos")
    assert lo * (1 - 1e-12) <= tlo <= 1.02 * lo, (tlo, lo)
    assert 0.99 * hi <= thi <= hi * (1 + 1e-12), (thi, hi)


def test_scan_and_bisection_reproduce_the_stored_c1_kappa(c1_links):
    res = search(c1_links, (4, 4, 4, 4), 1e-3, log=_quiet, stop_at_dip=False)
    with open(OUT) as fh:
        stored = json.load(fh)["c1"]
    assert res["kappa"] == pytest.approx(stored["kappa"], abs=1e-12)
    assert not res["target_unreachable"] and res["beyond_physical"]
    got = [(e["kappa"], e["ratio"]) for e in res["evaluations"]]
    want = [(e["kappa"], e["ratio"]) for e in stored["evaluations"]]
    assert len(got) == len(want)
    for (k1, r1), (k2, r2) in zip(got, want):
        assert k1 == pytest.approx(k2, abs=1e-12) and r1 == pytest.approx(r2, rel=1e-9)
    lo, hi, _ = extremes_dense(WilsonEO(c1_links, (4, 4, 4, 4), res["kappa"]))
    assert abs(math.log10(lo / hi / 1e-3)) <= 0.05


def test_bisection_with_lanczos_extremes_meets_the_target_by_dense_eigenvalues(c1_links):
    dims = (4, 4, 4, 4)
    U = flux_background(dims, 1, 1) @ c1_links
    target = 1e-4
    res = search(U, dims, target, log=_quiet, k_start=0.15, force_lanczos=True)
    assert not res["target_unreachable"]
    assert all(e["how"].startswith("lanczos") for e in res["evaluations"])
    lo, hi, _ = extremes_dense(WilsonEO(U, dims, res["kappa"]))
    # 0.05 from the bisection's stop, 0.01 for the Lanczos lambda_min (within 2%)
    assert abs(math.log10(lo / hi / target)) <= 0.06, (res["kappa"], lo / hi)


def test_dip_branch_finds_the_minimum_of_a_dense_grid(c1_links):
    dims = (4, 4, 4, 4)
    res = search(c1_links, dims, 1e-3, log=_quiet, stop_at_dip=True)
    assert res["target_unreachable"]
    grid = np.arange(0.140, 0.1601, 0.0025)
    ratios = []
    for k in grid:
        lo, hi, _ = extremes_dense(WilsonEO(c1_links, dims, float(k)))
        ratios.append(lo / hi)
    i = int(np.argmin(ratios))
    assert 0 < i < len(grid) - 1          # the grid brackets the dip
    assert res["ratio"] <= 1.002 * ratios[i], (res["ratio"], ratios[i])
    assert abs(res["kappa"] - grid[i]) <= 0.0025
