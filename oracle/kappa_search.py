"""Choose each workload's hopping parameter kappa with the oracle (writes synth/kappa.json).

The workloads ask for lambda_min(M)/lambda_max(M) of M = A^dag A near a target ratio.
Rule: scan kappa upward from 0.10 (0.15 for the batch members, whose rough links put the
critical kappa near 0.2; step 0.01, 0.05 above 0.30) to the first kappa whose
ratio is below the target, then bisect between the last two scan points until
|log10(ratio / target)| <= 0.05.  If the ratio turns upward before reaching the target (a
local minimum of the ratio near the critical kappa), the minimum is refined by golden-section
search; if the refined minimum lies below the target the left flank is bisected to the target,
otherwise the minimum is kept and the target is recorded as unreachable on this configuration.
The workloads of the paper's kind sit near the critical kappa (section 3), so they stop at that
dip.  The 4^4 correctness workload asks only for the ratio (its dip misses it by far): its scan
goes on past the dip to the first crossing, beyond the physical window (stop_at_dip=False).
The extreme eigenvalues come from a dense eigvalsh while 12*Vh <= 3072, otherwise from a plain
Lanczos run (three-term recurrence, Ritz values of T) stopped when the residual bound of the
lowest Ritz pair, beta_i |s_i|, is below 2% of that Ritz value.

Usage: python -m oracle.kappa_search c1 c2 ...
This is a data-preparation script of the oracle: its output is an input of the workloads.
"""
import json
import math
import os
import sys
import time

import numpy as np
from scipy.linalg import eigh_tridiagonal, eigvalsh_tridiagonal

from oracle.wilson import WilsonEO, dense, flat, matvec_M

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(os.path.dirname(HERE), "synth", "kappa.json")


def extremes_dense(op):
    mv = matvec_M(op)
    M = dense(mv, 12 * op.Vh)
    lam = np.linalg.eigvalsh(0.5 * (M + M.conj().T))
    return float(lam[0]), float(lam[-1]), "dense"


def extremes_lanczos(op, seed=12345, rtol=2e-2, max_iter=8000, log=None):
    """Plain Lanczos from a random start; stop when the lowest Ritz pair has residual <= rtol * theta."""
    mv = matvec_M(op)
    rng = np.random.default_rng(seed)
    N = 12 * op.Vh
    v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    v /= np.linalg.norm(v)
    v_prev = np.zeros_like(v)
    b_prev = 0.0
    a_list, b_list = [], []
    lo_hist = []
    lo = hi = None
    for i in range(1, max_iter + 1):
        f = mv(v) - b_prev * v_prev
        a = float(np.vdot(v, f).real)
        f -= a * v
        b = float(np.linalg.norm(f))
        a_list.append(a)
        b_list.append(b)
        if i % 50 == 0 or b < 1e-12:
            th, S = eigh_tridiagonal(np.array(a_list), np.array(b_list[:-1]), select="i", select_range=(0, 0))
            lo = float(th[0])
            hi = float(eigvalsh_tridiagonal(np.array(a_list), np.array(b_list[:-1]), select="i",
                                            select_range=(i - 1, i - 1))[0])
            resid = abs(b * S[-1, 0])
            lo_hist.append((i, lo))
            if log:
                log(f"    lanczos it={i} theta_min={lo:.6e} resid={resid:.2e} theta_max={hi:.6e}")
            if resid <= rtol * lo or b < 1e-12:
                break
        v_prev, v = v, f / b
        b_prev = b
    return lo, hi, f"lanczos({i})"


def ratio_of(links, dims, kappa, t_bc=-1, log=None, force_lanczos=False):
    op = WilsonEO(links, dims, kappa, t_bc=t_bc)
    if 12 * op.Vh <= 3072 and not force_lanczos:
        lo, hi, how = extremes_dense(op)
    else:
        lo, hi, how = extremes_lanczos(op, log=log)
    return lo / hi, lo, hi, how


def search(links, dims, target, t_bc=-1, log=print, k_start=0.10, stop_at_dip=True, force_lanczos=False):
    evals = []

    def f(k):
        r, lo, hi, how = ratio_of(links, dims, k, t_bc, log=None, force_lanczos=force_lanczos)
        evals.append(dict(kappa=k, ratio=r, lambda_min=lo, lambda_max=hi, how=how))
        log(f"  kappa={k:.6f} ratio={r:.4e} ({how})")
        return math.log10(r / target), r, lo, hi

    hist = []
    k_prev, k = None, k_start
    g, r, lo, hi = f(k)
    hist.append((k, g, r, lo, hi))
    unreachable = False
    while g > 0:
        k_prev = k
        k = round(k + (0.01 if k < 0.30 - 1e-12 else 0.05), 6)
        if k > 2.0:
            raise RuntimeError("no kappa below 2.0 reaches the target ratio")
        g, r, lo, hi = f(k)
        hist.append((k, g, r, lo, hi))
        if stop_at_dip and g > 0 and len(hist) >= 3 and hist[-2][1] < hist[-3][1] and hist[-2][1] < g:
            # the ratio turned upward: refine the local minimum between the last three points
            a, b = hist[-3][0], hist[-1][0]
            phi = (math.sqrt(5.0) - 1.0) / 2.0
            c, d = b - phi * (b - a), a + phi * (b - a)
            fc, fd = f(c), f(d)
            while b - a > 1e-3 and fc[0] > 0 and fd[0] > 0:
                if fc[0] < fd[0]:
                    b, d, fd = d, c, fc
                    c = b - phi * (b - a)
                    fc = f(c)
                else:
                    a, c, fc = c, d, fd
                    d = a + phi * (b - a)
                    fd = f(d)
            kmin, fmin = (c, fc) if fc[0] < fd[0] else (d, fd)
            if fmin[0] > 0.05:
                g, r, lo, hi = fmin
                unreachable = True
                return dict(kappa=kmin, ratio=r, lambda_min=lo, lambda_max=hi, target=target,
                            target_unreachable=True, beyond_physical=bool(kmin > 0.25), evaluations=evals)
            # the dip reaches the target: bisect its left flank
            k_prev, k, g = hist[-3][0], kmin, fmin[0]
            r, lo, hi = fmin[1], fmin[2], fmin[3]
            break
    if k_prev is None:
        raise RuntimeError(f"target already met at kappa = {k_start}")
    a, b = k_prev, k           # f(a) > 0 >= f(b)
    best = (abs(g), k, r, lo, hi)
    while abs(g) > 0.05:
        mid = 0.5 * (a + b)
        g, r, lo, hi = f(mid)
        if abs(g) < best[0]:
            best = (abs(g), mid, r, lo, hi)
        if g > 0:
            a = mid
        else:
            b = mid
        if b - a < 1e-7:
            break
    _, k, r, lo, hi = best
    return dict(kappa=k, ratio=r, lambda_min=lo, lambda_max=hi, target=target, target_unreachable=False,
                beyond_physical=bool(k > 0.25), evaluations=evals)


def main(names):
    from synth.configs import CONFIGS, make_links, batch_members
    table = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            table = json.load(fh)
    members = {c.name: c for c in batch_members()}
    for name in names:
        cfg = CONFIGS.get(name) or members[name]
        t0 = time.time()
        print(f"{name}: dims={cfg.dims} eps={cfg.eps} ape={cfg.ape_steps} target={cfg.ratio:g}", flush=True)
        U = make_links(cfg)
        # batch members (rough links, kappa_c near 0.2) start the scan higher
        res = search(U, cfg.dims, cfg.ratio, cfg.t_bc, k_start=0.15 if name.startswith("c4_") else 0.10,
                     stop_at_dip=name != "c1")
        res["seconds"] = round(time.time() - t0, 1)
        table[name] = res
        # re-read and merge so that concurrent searches of other workloads are kept
        if os.path.exists(OUT):
            with open(OUT) as fh:
                cur = json.load(fh)
            cur.update({name: res})
            table = cur
        with open(OUT, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        print(f"{name}: kappa={res['kappa']:.6f} ratio={res['ratio']:.3e} ({res['seconds']} s)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
