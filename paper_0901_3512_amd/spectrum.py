"""Extreme eigenvalues of M = A^dag A from the library's FP64 Lanczos, and a kappa search on them.

A workload's conditioning lambda_min / lambda_max of M (section 3; kappa near its critical value)
sets how many Lanczos and CG steps it needs.  At lattices the CPU cannot diagonalise, this
estimates the extremes on the GPU: a seed solve of one random right-hand side with a fixed m,
without reorthogonalisation, gives the Lanczos coefficients of Eq. (2); the extreme eigenvalues
of that tridiagonal T are the Ritz values.  Without reorthogonalisation the converged extreme
Ritz values are still eigenvalues of M (loss of orthogonality only repeats them), and the lowest
one carries the residual bound beta_m |s_m| of its Ritz vector.

The search takes the same steps as the CPU one the small workloads use: scan kappa upward
(step 0.01, 0.05 above 0.30) to the first kappa whose ratio is below the target and bisect to
|log10(ratio / target)| <= 0.05; if the ratio turns upward first (a dip near the critical kappa)
refine the dip by golden-section search, bisect its left flank if it reaches the target and
otherwise keep its minimum and record the target as unreachable.

Usage (on a GPU):  python -m paper_0901_3512_amd.spectrum --out synth/kappa.json c3 c3t c5 c5t
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch
from scipy.linalg import eigh_tridiagonal, eigvalsh_tridiagonal

from .seedcg import SeedCG


def extremes(links, dims, kappa, m, *, t_bc=-1, seed=1, keep=False):
    """Lanczos extremes of M at kappa from m FP64 steps on a random start (no reorthogonalisation).

    Returns dict(lo, hi, resid_lo, m, seconds) and, with keep=True, also the handle (whose basis
    holds the Lanczos vectors) and the Ritz coefficient vectors s_lo, s_hi of T."""
    dev = links.device
    s = SeedCG(links, dims, kappa, t_bc=t_bc, prec="fp64", m_max=m, reorth_k=0, past=0.0, tol=1e-300,
               autotune=False)
    Vh = int(np.prod(dims)) // 2
    g = torch.Generator(device=dev).manual_seed(seed)
    b = torch.randn((1, Vh, 4, 3), dtype=torch.complex128, device=dev, generator=g)
    t0 = time.perf_counter()
    _, rep = s.solve_seed(b)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    a, be = s.get_tridiag()
    a, be = np.array(a), np.array(be)
    k = len(a)
    th, S = eigh_tridiagonal(a, be[1:k], select="i", select_range=(0, 0))
    hi, Sh = eigh_tridiagonal(a, be[1:k], select="i", select_range=(k - 1, k - 1))
    out = dict(lo=float(th[0]), hi=float(hi[0]), resid_lo=float(abs(be[k] * S[-1, 0])), m=k, seconds=t)
    if keep:
        out.update(handle=s, s_lo=S[:, 0], s_hi=Sh[:, 0])
    else:
        s.close()
    return out


def search(links, dims, target, *, m, t_bc=-1, k_start=0.10, log=print):
    evals = []

    def f(k):
        e = extremes(links, dims, k, m, t_bc=t_bc)
        r = e["lo"] / e["hi"]
        evals.append(dict(kappa=k, ratio=r, lambda_min=e["lo"], lambda_max=e["hi"], resid_min=e["resid_lo"],
                          how=f"gpu-lanczos({e['m']})"))
        log(f"  kappa={k:.6f} ratio={r:.4e} lo={e['lo']:.4e} resid={e['resid_lo']:.1e} ({e['seconds']:.1f} s)")
        torch.cuda.empty_cache()
        return math.log10(r / target), r, e["lo"], e["hi"]

    def record(k, r, lo, hi, unreachable):
        return dict(kappa=k, ratio=r, lambda_min=lo, lambda_max=hi, target=target, target_unreachable=unreachable,
                    beyond_physical=bool(k > 0.25), evaluations=evals, estimator="gpu-lanczos", m=m)

    hist = []
    k_prev, k = None, k_start
    g, r, lo, hi = f(k)
    hist.append((k, g))
    if g <= 0:
        raise RuntimeError(f"target already met at kappa = {k_start}")
    while g > 0:
        k_prev = k
        k = round(k + (0.01 if k < 0.30 - 1e-12 else 0.05), 6)
        if k > 2.0:
            raise RuntimeError("no kappa below 2.0 reaches the target ratio")
        g, r, lo, hi = f(k)
        hist.append((k, g))
        if g > 0 and len(hist) >= 3 and hist[-2][1] < hist[-3][1] and hist[-2][1] < g:
            a, b = hist[-3][0], hist[-1][0]
            phi = (math.sqrt(5.0) - 1.0) / 2.0
            c, d = b - phi * (b - a), a + phi * (b - a)
            fc, fd = (c,) + f(c), (d,) + f(d)
            while b - a > 1e-3 and fc[1] > 0 and fd[1] > 0:
                if fc[1] < fd[1]:
                    b, d, fd = d, c, fc
                    c = b - phi * (b - a)
                    fc = (c,) + f(c)
                else:
                    a, c, fc = c, d, fd
                    d = a + phi * (b - a)
                    fd = (d,) + f(d)
            best = fc if fc[1] < fd[1] else fd
            if best[1] > 0.05:
                return record(best[0], best[2], best[3], best[4], True)
            k_prev, k, g = hist[-3][0], best[0], best[1]
            r, lo, hi = best[2], best[3], best[4]
            break
    a, b = k_prev, k
    best = (abs(g), k, r, lo, hi)
    while abs(g) > 0.05 and b - a > 1e-7:
        mid = 0.5 * (a + b)
        g, r, lo, hi = f(mid)
        if abs(g) < best[0]:
            best = (abs(g), mid, r, lo, hi)
        if g > 0:
            a = mid
        else:
            b = mid
    _, k, r, lo, hi = best
    return record(k, r, lo, hi, False)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("names", nargs="+")
    ap.add_argument("--out", required=True, help="JSON table of kappas to merge the results into")
    ap.add_argument("--m", type=int, default=0, help="Lanczos steps per estimate (0: by lattice size)")
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    from synth.configs import CONFIGS, make_links
    dev = torch.device("cuda:0")
    for name in args.names:
        cfg = CONFIGS[name]
        m = args.m or (1000 if cfg.volume > 1_000_000 else 1500)
        t0 = time.time()
        print(f"{name}: dims={cfg.dims} eps={cfg.eps} flux={cfg.flux} target={cfg.ratio:g} m={m}", flush=True)
        U = torch.from_numpy(make_links(cfg)).to(dev)
        res = search(U, cfg.dims, cfg.ratio, m=m, t_bc=cfg.t_bc)
        res["seconds"] = round(time.time() - t0, 1)
        del U
        torch.cuda.empty_cache()
        table = {}
        if os.path.exists(args.out):
            with open(args.out) as fh:
                table = json.load(fh)
        table[name] = res
        with open(args.out, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        print(f"{name}: kappa={res['kappa']:.6f} ratio={res['ratio']:.3e} unreachable={res['target_unreachable']} "
              f"({res['seconds']} s)", flush=True)


if __name__ == "__main__":
    main()
