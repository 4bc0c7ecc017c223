"""Benchmark: RHS/s of Seed-CG at an FP64 relative residual of 1e-10, learned + mixed against plain FP64
Seed-CG on the same lattice, and the D^dag D stencil rate.

One step = the whole hot path on one batch of right-hand sides of one configuration: Algorithm 1 on
RHS 1 (Lanczos run past convergence, periodic reorthogonalisation, Galerkin seeding of the others
through the LU of T), then CG from the seeded guesses on every right-hand side, until each one has an
FP64 true relative residual <= tol.  Inputs are resident in HBM before the timed region.

The headline line (default): `value` is the learned + mixed form, timed per step as
  solve_seed (FP64 Algorithm 1; FP64 basis, plus an FP32 copy of it that only the periodic
    reorthogonalisation reads where HBM holds both: --basis)
  + train_precond (the learned K K^dag, 2000 Adam steps on the seed solve's Ritz vectors and
    residuals, then judged against plain CG on RHS 2)
  + solve_rest (FP32 CG with FP64 reliable updates; PCG with K and the 16 lowest Ritz vectors of the
    seed basis deflated when K won the judge, otherwise plain CG, deflated only when the judge priced
    deflation cheaper);
`vs_baseline` is that RHS/s over plain FP64 Seed-CG's (solve_seed + solve_rest, all FP64) on the same
lattice, right-hand sides and GPU, timed in the same run: the comparison the metric names.
Default workload: 24^3 x 48 on the topological flux background at lambda_min/lambda_max = 1.1e-5,
12 point + 12 Z2 sources, k = 10 (--config c5t: 32^3 x 64 at 9.7e-7, 12 point sources).

--form fp64|mixed|mixed_cg|mixed_bf16: one form only (the earlier single-form line, with the
same-lattice comparisons); --config c4: the batched workload (64 configurations of {8^4, 8^3 x 16,
12^3 x 24, 12^4}, one batch call per step); --sweep: RHS 1's cost and RHS 2's CG iterations
against k and the past-convergence factor.

Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
METRIC = "RHS/s at FP64 rel. residual 1e-10 (learned+mixed vs plain Seed-CG); D†D GB/s"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3t", help="c3t (default), c5t, c2, c2t, c4 (the batch), or one batch member c4_00 ... c4_63")
    ap.add_argument("--form", default="metric",
                    help="metric (learned + mixed against plain FP64, default) or one form: fp64|mixed|mixed_cg|mixed_bf16")
    ap.add_argument("--prec", default=None, help="with --form: override the workload precision")
    ap.add_argument("--train-steps", type=int, default=2000, help="Adam steps of the learned K per step")
    ap.add_argument("--deflate-k", type=int, default=16, help="Ritz vectors deflated in the learned form's (P)CG")
    ap.add_argument("--ref-steps", type=int, default=5, help="timed steps of the plain FP64 reference (at most --steps)")
    ap.add_argument("--m-max", type=int, default=0,
                    help="Krylov basis capacity (0: the metric's line sizes it by the GPU's memory, --form grows it as the run needs)")
    ap.add_argument("--basis", default="auto", choices=("auto", "fp64", "fp32", "reorth"),
                    help="the Krylov basis of the learned + mixed form (or of --form): FP64; FP32; FP64 plus an FP32 copy "
                         "read only by the reorthogonalisation; auto = reorth where HBM holds both at the capacity, "
                         "else FP64 (--form: the precision's own basis)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=40, help="Lanczos steps in the oracle sample")
    ap.add_argument("--sample-every", type=int, default=7,
                    help="stencil launches per timed sample (coprime to the 4 launches of one M, so every launch kind is sampled)")
    ap.add_argument("--mbench", type=int, default=200, help="back-to-back M applications for D^dag D GB/s")
    ap.add_argument("--batch-n", type=int, default=64, help="c4: number of batch members (the workload has 64)")
    ap.add_argument("--deflate", type=int, default=0, help="deflated CG with this many Ritz vectors (0: plain CG)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the same-lattice comparison runs (mixed precision, and learned K with --learned)")
    ap.add_argument("--learned", action="store_true", help="compare also the learned preconditioner (2000 Adam steps)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 1 GiB device copy first (reference for the HBM byte counters)")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark line: the cost of RHS 1 and the CG iterations of RHS 2 against the "
                         "reorthogonalisation frequency k and the past-convergence factor (FP64, two right-hand sides)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    from __graft_entry__ import _built, build
    if not _built():
        build()
    from paper_0901_3512_amd import SeedCG
    from synth.configs import CONFIGS, make_links, make_sources, kappa_for

    if args.config == "c4":
        return bench_batch(args)   # generates its inputs in worker processes before any GPU call
    if args.form == "metric" and not args.sweep:
        return bench_metric(args)
    if args.config.startswith("c4_"):   # one member of the batched workload on its own
        from synth.configs import batch_members
        cfg = {m.name: m for m in batch_members()}[args.config]
    else:
        cfg = CONFIGS[args.config]
    prec = args.prec or (args.form if args.form != "metric" else cfg.prec)
    dev = torch.device("cuda:0")
    t_gen = time.time()
    U = make_links(cfg)
    phi = make_sources(cfg)
    kappa = kappa_for(cfg)
    log(f"inputs {cfg.name} dims={cfg.dims} kappa={kappa} nrhs={cfg.nrhs} ({time.time() - t_gen:.1f} s)")
    Ud = torch.from_numpy(U).to(dev)
    phid = torch.from_numpy(phi).to(dev)
    # one form's basis: as --basis asks (auto: the FP64 basis of an FP64 Lanczos, or the FP32 one)
    basis = {"auto": False, "fp64": False, "fp32": True, "reorth": "reorth"}[args.basis]
    solver = SeedCG(Ud, cfg.dims, kappa, t_bc=cfg.t_bc, prec=prec, reorth_k=cfg.reorth_k, past=cfg.past,
                    tol=cfg.tol, reliable_every=cfg.reliable_every, deflate=args.deflate, basis_fp32=basis, m_max=args.m_max)
    B = solver.apply_A(phid, dagger=True)   # b = A^dag phi (input preparation, not timed)
    if args.sweep:
        return sweep(cfg, Ud, kappa, B)
    nrhs = B.shape[0]
    torch.cuda.synchronize()

    def step():
        X = torch.zeros_like(B)
        X, rs = solver.solve_seed(B, X)
        X, rr = solver.solve_rest(B, X)
        return X, rs, rr

    for w in range(args.warmup):
        _, rs, rr = step()
        log(f"warmup {w}: m={rs['m']} i_conv={rs['i_conv']} seed {rs['t_seed_s']:.3f}s rest {rr['t_rest_s']:.3f}s "
            f"iters={rr['iters']}")

    if args.copy_probe:
        copy_probe()   # marks the start of the timed region in a counter trace
    solver.set_timing(args.sample_every, 8192)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reports = []
    solved = 0
    for k in range(args.steps):
        X, rs, rr = step()
        reports.append((rs, rr))
        solved += sum(1 for r in rr["true_relres"] if r <= cfg.tol)
        log(f"step {k}: m={rs['m']} seed {rs['t_seed_s']:.3f}s rest {rr['t_rest_s']:.3f}s "
            f"max relres {max(rr['true_relres']):.2e}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = solver.get_timing()
    solver.set_timing(0, 0)
    elapsed = t1 - t0
    value = solved / elapsed

    # D^dag D rate: back-to-back applications of M inside the library, timed with events (FP64, and the
    # CG's inner precision for the mixed forms)
    V = int(np.prod(cfg.dims))
    dd = dagger_d(solver, prec, nrhs, args.mbench) if args.mbench > 0 else None
    # roofline of the dominant kernel (the Wilson hop), measured live over the timed region
    hop_ms = tm["ms"] / max(tm["launches"], 1)
    hop_bytes = tm["bytes"] / max(tm["launches"], 1)
    achieved = hop_bytes / (hop_ms * 1e-3) / 1e9 if tm["launches"] else None
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                "traffic": measured_traffic(cfg, prec),
                "kernel": "even-odd Wilson hop (hop_split_kernel, or the launch shape the autotuner picked), fused epilogues", "launches_sampled": tm["launches"],
                "avg_launch_us": hop_ms * 1e3, "avg_launch_bytes": hop_bytes}
    if prec == "fp64" and achieved:
        # the same launches priced with whole 3x3 links (18 reals) instead of the two rows (12 reals)
        # the stencil reads for special-unitary fields: 8 links per output site, 6 reals more each
        extra = (V // 2) * 8 * 6 * 8.0
        roofline["achieved_18real_links"] = (hop_bytes + extra) / (hop_ms * 1e-3) / 1e9

    compare = None
    if not args.no_compare:
        compare = compare_forms(args, cfg, Ud, kappa, B, value, prec, phid)
    copy_gbs = copy_rate()
    probes = roofline_probes()
    with_achievable(roofline, probes)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, U, phi, kappa, reports[-1], args.cpu_iters)

    rs, rr = reports[-1]
    result = {
        "metric": METRIC, "value": value, "unit": "RHS/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == "fp64" else f"f32+f64({prec})",
        "data": "synthetic",
        "config": {"workload": f"Seed-CG {prec}, Wilson even-odd normal system M = A^dag A on "
                               f"{'x'.join(map(str, cfg.dims))}, {cfg.nrhs} RHS, tol {cfg.tol:g}, k={cfg.reorth_k}",
                   "name": cfg.name, "lattice": list(cfg.dims), "kappa": kappa, "nrhs": nrhs,
                   "reorth_k": cfg.reorth_k, "past_factor": cfg.past, "tol": cfg.tol, "precision": prec,
                   "deflate": args.deflate, "basis": args.basis},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {"m": rs["m"], "i_conv": rs["i_conv"], "seed_status": rs["seed_status"],
                   "t_seed_s": rs["t_seed_s"], "t_rest_s": rr["t_rest_s"], "cg_iters": rr["iters"],
                   "max_true_relres": max(rr["true_relres"]), "dagger_d": dd,
                   "hop_launches_total": tm["seen"], "compare": compare,
                   "device_copy_gbs": copy_gbs, "roofline_probes": probes},
    }
    print(json.dumps(result), flush=True)


FMT_NAMES = {0: "fp64", 1: "fp32", 2: "fp32 (bf16 links)", 3: "fp64 (two-row links)", 4: "fp32 (two-row links)"}


def dagger_d(solver, prec, nrhs, reps):
    """D^dag D rate of back-to-back M applications timed with events inside the library: FP64 for one
    vector and for the nrhs - 1 of the CG; for the mixed forms also the CG's inner precision."""
    out = {}
    forms = [("fp64", False)] + ([("inner", True)] if prec != "fp64" else [])
    for name, inner in forms:
        for nv in sorted({1, max(1, nrhs - 1)}):
            t = solver.time_M(inner=inner, nvec=nv, reps=reps)
            out[f"{name}_nvec{nv}"] = {"gbs": t["bytes"] / (t["ms"] * 1e-3) / 1e9,
                                       "gbs_18real_links": t["bytes_18real"] / (t["ms"] * 1e-3) / 1e9,
                                       "us_per_M": t["ms"] * 1e3, "links": FMT_NAMES.get(t["fmt"], t["fmt"]),
                                       "frac_hbm": t["bytes"] / (t["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


def dominant_kind(kinds):
    """The stencil launch kind with the largest sampled time."""
    if not kinds:
        return None
    k = max(kinds, key=lambda r: r["ms"])
    return dict(k, avg_us=1e3 * k["ms"] / k["launches"], avg_bytes=k["bytes"] / k["launches"],
                gbs=k["bytes"] / (k["ms"] * 1e-3) / 1e9, name=kind_name(k))


_FMT_TYPES = {0: ("double", "double"), 1: ("float", "float"), 2: ("float", "scg::bf16link"),
              3: ("double", "scg::su3rows<double>"), 4: ("float", "scg::su3rows<float>")}


def kind_kernel(k):
    """The kernel a stencil launch kind runs, as rocprofv3 names it (the production launch shapes)."""
    t, lt = _FMT_TYPES.get(int(k["fmt"]), ("?", "?"))
    cgu = "true" if k["fused"] else "false"
    tps, vb = int(k["tps"]), int(k["vb"])
    if tps == 8:
        return f"scg::hop_split_kernel<{t}, {lt}, {vb}, {cgu}>"
    if tps == 9:
        return f"scg::hop_plane_kernel<{t}, {lt}, {vb}, {cgu}>"
    if tps == 10:
        return f"scg::hop_quad_kernel<{t}, {lt}, {cgu}>"
    if tps == 11:
        return f"scg::hop_stream_kernel<{t}, {lt}, {vb}, {cgu}>"
    if tps == 12:
        return f"scg::hop_quad_nt_kernel<{t}, {lt}, {cgu}>"
    return f"scg::hop (launch shape tps {tps}, vb {vb})"


def kind_tag(k):
    fam = {8: "split", 9: "plane", 10: "quad", 11: "stream", 12: "quadnt"}.get(int(k["tps"]), f"tps{int(k['tps'])}")
    return f"{FMT_NAMES.get(int(k['fmt']), 'x').split()[0]}_{fam}_vb{int(k['vb'])}{'_cgu' if k['fused'] else ''}"


def kind_name(k):
    return (f"{kind_kernel(k)}: {FMT_NAMES.get(int(k['fmt']), k['fmt'])}, {int(k['nvec'])} vector(s) per launch"
            f"{', CG update fused' if k['fused'] else ''}")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_metric(args):
    """The metric's own comparison: learned + mixed Seed-CG against plain FP64 Seed-CG, same lattice."""
    import numpy as np
    import torch
    from paper_0901_3512_amd import SeedCG
    from synth.configs import CONFIGS, make_links, make_sources, kappa_for
    cfg = CONFIGS[args.config]
    dev = torch.device("cuda:0")
    t_gen = time.time()
    U = make_links(cfg)
    phi = make_sources(cfg)
    kappa = kappa_for(cfg)
    log(f"inputs {cfg.name} dims={cfg.dims} kappa={kappa} nrhs={cfg.nrhs} ({time.time() - t_gen:.1f} s)")
    Ud = torch.from_numpy(U).to(dev)
    phid = torch.from_numpy(phi).to(dev)
    # the same basis capacity for both forms (FP64 basis in both): 1000 vectors, or what 60% of the
    # GPU's memory holds at this lattice (the two forms run one after the other, never both at once)
    vec_bytes = cfg.volume // 2 * 12 * 16
    m_max = args.m_max or min(1000, int(0.6 * torch.cuda.get_device_properties(0).total_memory // vec_bytes))
    common = dict(t_bc=cfg.t_bc, reorth_k=cfg.reorth_k, past=cfg.past, tol=cfg.tol, reliable_every=cfg.reliable_every,
                  m_max=m_max)
    # the value form's basis: the FP64 basis (the seeding keeps its full gain) plus an FP32 copy that
    # halves the reorthogonalisation's reads, where 60% of the GPU's memory holds both at the capacity
    basis = args.basis
    if basis == "auto":
        hbm = torch.cuda.get_device_properties(0).total_memory
        basis = "reorth" if m_max * vec_bytes * 3 // 2 <= 0.6 * hbm else "fp64"
    val = SeedCG(Ud, cfg.dims, kappa, prec="mixed_cg", deflate=args.deflate_k,
                 basis_fp32={"fp64": False, "fp32": True, "reorth": "reorth"}[basis], **common)
    B = val.apply_A(phid, dagger=True)   # b = A^dag phi (input preparation, not timed)
    nrhs = B.shape[0]

    def step_val():
        X = torch.zeros_like(B)
        X, rs = val.solve_seed(B, X)
        t = time.perf_counter()
        tr = val.train_precond(steps=args.train_steps, n_ritz=4, n_lanczos=12, lr=2e-4)
        tr["t_train_and_judge_s"] = time.perf_counter() - t
        val.use_precond(tr["accepted"])
        X, rr = val.solve_rest(B, X)
        return rs, tr, rr

    def step_ref():
        X = torch.zeros_like(B)
        X, rs = ref.solve_seed(B, X)
        X, rr = ref.solve_rest(B, X)
        return rs, rr

    for w in range(args.warmup):
        rs, tr, rr = step_val()
        log(f"warmup {w}: m={rs['m']} i_conv={rs['i_conv']} seed {rs['t_seed_s']:.2f}s train {tr['t_train_s']:.2f}s "
            f"({tr['choice']}, judge {tr['judge_iters']}, predicted {tr['predicted_s']}) rest {rr['t_rest_s']:.2f}s "
            f"iters={rr['iters']}")
    if args.copy_probe:
        copy_probe()   # marks the start of the timed region in a counter trace

    # the value: learned + mixed, every step including the training of K
    val.set_timing(args.sample_every, 16384)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solved, t_train, last = 0, 0.0, None
    for k in range(args.steps):
        rs, tr, rr = step_val()
        last = (rs, tr, rr)
        t_train += tr["t_train_s"]
        solved += sum(1 for r in rr["true_relres"] if r <= cfg.tol)
        log(f"step {k}: m={rs['m']} seed {rs['t_seed_s']:.2f}s train {tr['t_train_s']:.2f}s (+judge "
            f"{tr['t_train_and_judge_s'] - tr['t_train_s']:.2f}s, {tr['choice']}, plain CG deflates: "
            f"{tr['plain_cg_deflates']}) rest {rr['t_rest_s']:.2f}s max relres {max(rr['true_relres']):.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kinds = val.get_timing_kinds()
    val.set_timing(0, 0)
    value = solved / elapsed
    dd = dagger_d(val, "mixed_cg", nrhs, args.mbench) if args.mbench > 0 else None
    val.close()
    del val
    torch.cuda.empty_cache()

    # the baseline: plain FP64 Seed-CG on the same inputs
    ref = SeedCG(Ud, cfg.dims, kappa, prec="fp64", **common)
    rs_w, rr_w = step_ref()
    log(f"reference warmup: m={rs_w['m']} seed {rs_w['t_seed_s']:.2f}s rest {rr_w['t_rest_s']:.2f}s iters={rr_w['iters']}")
    nref = max(1, min(args.steps, args.ref_steps))
    ref.set_timing(args.sample_every, 16384)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solved_ref, last_ref = 0, None
    for k in range(nref):
        rs_r, rr_r = step_ref()
        last_ref = (rs_r, rr_r)
        solved_ref += sum(1 for r in rr_r["true_relres"] if r <= cfg.tol)
    torch.cuda.synchronize()
    elapsed_ref = time.perf_counter() - t0
    kinds_ref = ref.get_timing_kinds()
    ref.set_timing(0, 0)
    value_ref = solved_ref / elapsed_ref
    log(f"learned+mixed {value:.3f} RHS/s, plain FP64 {value_ref:.3f} RHS/s ({value / value_ref:.2f}x)")
    ref.close()

    dom = dominant_kind(kinds)
    traffic = measured_traffic(cfg, kind_tag(dom), kind_kernel(dom)) if dom else None
    roofline = {"bound": "hbm", "achieved": dom["gbs"] if dom else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dom["gbs"] / HBM_PEAK_GBS if dom else None, "traffic": traffic,
                "kernel": dom["name"] if dom else None,
                "launches_sampled": int(dom["launches"]) if dom else 0, "avg_launch_us": dom["avg_us"] if dom else None,
                "avg_launch_bytes": dom["avg_bytes"] if dom else None,
                "note": "the sampled launch kind with the largest stencil time in the timed learned + mixed steps; "
                        "algorithmic bytes (links once per launch in the stored format, every spinor operand once)"}
    probes = roofline_probes()
    with_achievable(roofline, probes)
    # the same figures for the next launch kinds by stencil time (the dominant one can change with a
    # small shift in the split between the Lanczos steps and the CG)
    runners_up = []
    for k in sorted(kinds, key=lambda r: -r["ms"])[1:3]:
        d = dominant_kind([k])
        runners_up.append(with_achievable({
            "kernel": d["name"], "unit": "GB/s", "achieved": d["gbs"], "frac": d["gbs"] / HBM_PEAK_GBS,
            "traffic": measured_traffic(cfg, kind_tag(d), kind_kernel(d)), "launches_sampled": int(d["launches"]),
            "avg_launch_us": d["avg_us"], "avg_launch_bytes": d["avg_bytes"], "stencil_ms_sampled": d["ms"]}, probes))
    roofline["runners_up"] = runners_up
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, U, phi, kappa, last_ref, min(args.cpu_iters, 10 if cfg.volume > 300_000 else 40))
    rs, tr, rr = last
    rs_r, rr_r = last_ref
    result = {
        "metric": METRIC, "value": value, "unit": "RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": value / value_ref, "dtype": "f64+f32 (learned + mixed)", "data": "synthetic",
        "config": {"workload": f"learned + mixed Seed-CG against plain FP64 Seed-CG, Wilson even-odd M = A^dag A on "
                               f"{'x'.join(map(str, cfg.dims))}"
                               f"{' with a topological flux background' if cfg.flux else ''}, "
                               f"lambda_min/lambda_max {cfg.ratio:g}, {nrhs} RHS, tol {cfg.tol:g}, k={cfg.reorth_k}",
                   "name": cfg.name, "lattice": list(cfg.dims), "kappa": kappa, "nrhs": nrhs, "reorth_k": cfg.reorth_k,
                   "past_factor": cfg.past, "tol": cfg.tol, "train_steps": args.train_steps,
                   "deflated_ritz_vectors": args.deflate_k, "m_max": m_max,
                   "learned_mixed_basis": {"fp64": "FP64", "fp32": "FP32",
                                           "reorth": "FP64, FP32 copy for the reorthogonalisation"}[basis]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {
            "vs_baseline_is": "learned + mixed RHS/s (training counted) over plain FP64 Seed-CG RHS/s on the same lattice, "
                              "inputs and GPU, timed in the same run",
            "plain_fp64": {"rhs_per_s": value_ref, "steps": nref, "ms_per_step": 1e3 * elapsed_ref / nref, "m": rs_r["m"],
                           "i_conv": rs_r["i_conv"], "t_seed_s": rs_r["t_seed_s"], "t_rest_s": rr_r["t_rest_s"],
                           "cg_iters": rr_r["iters"], "max_true_relres": max(rr_r["true_relres"]),
                           "dominant_stencil": dominant_kind(kinds_ref)},
            "learned_mixed": {"rhs_per_s": value, "rhs_per_s_without_training": solved / max(elapsed - t_train, 1e-9),
                              "t_train_s_per_step": t_train / args.steps, "m": rs["m"], "i_conv": rs["i_conv"],
                              "t_seed_s": rs["t_seed_s"], "t_rest_s": rr["t_rest_s"], "cg_iters": rr["iters"],
                              "max_true_relres": max(rr["true_relres"]), "training": tr},
            "stencil_kinds": kinds, "dagger_d": dd, "device_copy_gbs": copy_rate(), "roofline_probes": probes,
        },
    }
    print(json.dumps(result), flush=True)


def compare_forms(args, cfg, Ud, kappa, B, value_ref, prec_ref, phid):
    """The same lattice and right-hand sides solved by the other forms of the method, timed the same
    way (1 warmup, then args.steps solves): traditional repeated seeding; batched plain CG from zero
    on every right-hand side (no seeding); in FP64, the indefinite
    formulation (A x = phi through gamma5 A, seeded with the QR of the Lanczos matrix, finished by
    MINRES; its residual is that of A x = phi, and the normal-equation residual of its solutions is
    reported beside it); mixed precision (FP32 basis and CG), FP64 Lanczos with FP32 CG, and with
    --learned the learned K + mixed (training on the
    seed solve's Ritz and basis vectors is part of every step)."""
    import torch
    from paper_0901_3512_amd import SeedCG
    out = {"reference": {"form": prec_ref, "rhs_per_s": value_ref}}
    forms = [("mixed", False), ("mixed_cg", False)] + ([("mixed", True)] if args.learned else [])
    # the paper's comparison: traditional repeated seeding (each system's own Lanczos to convergence)
    s = SeedCG(Ud, cfg.dims, kappa, t_bc=cfg.t_bc, prec=prec_ref, reorth_k=cfg.reorth_k, tol=cfg.tol,
               reliable_every=cfg.reliable_every)
    s.solve_repeated(B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solved = 0
    for _ in range(args.steps):
        _, rr = s.solve_repeated(B)
        solved += sum(1 for r in rr["true_relres"] if r <= cfg.tol)
    torch.cuda.synchronize()
    v = solved / (time.perf_counter() - t0)
    out["repeated_seeding_" + prec_ref] = {"rhs_per_s": v, "vs_reference": v / value_ref, "iters": rr["iters"]}
    log(f"compare repeated seeding: {v:.2f} RHS/s ({v / value_ref:.2f}x)")
    s.close()
    # no seeding at all: batched CG on every right-hand side from x0 = 0 (what the method must beat)
    s = SeedCG(Ud, cfg.dims, kappa, t_bc=cfg.t_bc, prec=prec_ref, reorth_k=cfg.reorth_k, tol=cfg.tol,
               reliable_every=cfg.reliable_every)
    s.solve_rest(B, torch.zeros_like(B))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solved = 0
    for _ in range(args.steps):
        _, rr = s.solve_rest(B, torch.zeros_like(B))
        solved += sum(1 for r in rr["true_relres"] if r <= cfg.tol)
    torch.cuda.synchronize()
    v = solved / (time.perf_counter() - t0)
    out["plain_cg_" + prec_ref] = {"rhs_per_s": v, "vs_reference": v / value_ref, "iters": rr["iters"]}
    log(f"compare plain CG from zero: {v:.2f} RHS/s ({v / value_ref:.2f}x)")
    s.close()
    if prec_ref == "fp64":
        s = SeedCG(Ud, cfg.dims, kappa, t_bc=cfg.t_bc, prec="fp64", reorth_k=cfg.reorth_k, past=cfg.past, tol=cfg.tol)
        X, _ = s.solve_indefinite(phid)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solved = 0
        for _ in range(args.steps):
            X, ri = s.solve_indefinite(phid)
            solved += sum(1 for r in ri["true_relres"] if r <= cfg.tol)
        torch.cuda.synchronize()
        v = solved / (time.perf_counter() - t0)
        MX = s.apply_M(X)
        nres = (torch.linalg.vector_norm((B - MX).reshape(B.shape[0], -1), dim=1)
                / torch.linalg.vector_norm(B.reshape(B.shape[0], -1), dim=1))
        out["indefinite_qr_fp64"] = {"rhs_per_s": v, "vs_reference": v / value_ref, "m": ri["m"], "i_conv": ri["i_conv"],
                                     "iters": ri["iters"], "max_relres_A": max(ri["true_relres"]),
                                     "max_relres_normal": float(nres.max()), "t_seed_s": ri["t_seed_s"],
                                     "t_rest_s": ri["t_rest_s"]}
        log(f"compare indefinite (QR seeding of gamma5 A): {v:.2f} RHS/s ({v / value_ref:.2f}x)")
        s.close()
    for prec, learned in forms:
        s = SeedCG(Ud, cfg.dims, kappa, t_bc=cfg.t_bc, prec=prec, reorth_k=cfg.reorth_k, past=cfg.past, tol=cfg.tol,
                   reliable_every=cfg.reliable_every)
        tr = None

        def step():
            nonlocal tr
            X = torch.zeros_like(B)
            X, _ = s.solve_seed(B, X)
            if learned:
                tr = s.train_precond(steps=2000, n_ritz=8, n_lanczos=8, lr=1e-3)
                s.use_precond(True)
            X, rr = s.solve_rest(B, X)
            return rr
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solved = 0
        for _ in range(args.steps):
            rr = step()
            solved += sum(1 for r in rr["true_relres"] if r <= cfg.tol)
        torch.cuda.synchronize()
        v = solved / (time.perf_counter() - t0)
        key = "learned+" + prec if learned else prec
        out[key] = {"rhs_per_s": v, "vs_reference": v / value_ref, "cg_iters": rr["iters"],
                    "max_true_relres": max(rr["true_relres"])}
        if learned and tr:
            out[key]["training"] = tr
        log(f"compare {key}: {v:.2f} RHS/s ({v / value_ref:.2f}x)")
        s.close()
    return out


def sweep(cfg, Ud, kappa, B):
    """The trade-offs of the first right-hand side, with one extra right-hand side as in the paper's
    own test (Table 1: time of RHS 1 against k; Figures 1-2: CG of RHS 2 against m and k).
    For every setting: one untimed solve, then solve_seed timed on RHS 1 (Lanczos past convergence,
    reorthogonalisation, seeding of RHS 2), then CG on RHS 2 from its seeded guess.  Standard CG
    on RHS 2 from zero is the reference."""
    import torch
    from paper_0901_3512_amd import SeedCG
    B2 = B[:2].contiguous()

    def make(k, past):
        return SeedCG(Ud, cfg.dims, kappa, t_bc=cfg.t_bc, prec="fp64", reorth_k=k, past=past, tol=cfg.tol)

    s = make(cfg.reorth_k, cfg.past)
    _, rr = s.solve_rest(B2[1:], torch.zeros_like(B2[1:]))
    std = rr["iters"][0]
    del s

    def one(k, past):
        s = make(k, past)
        X, _ = s.solve_seed(B2, torch.zeros_like(B2))
        s.solve_rest(B2, X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, rs = s.solve_seed(B2, torch.zeros_like(B2))
        torch.cuda.synchronize()
        t_seed = time.perf_counter() - t0
        X, rr = s.solve_rest(B2, X)
        out = {"k": k, "past": past, "m": rs["m"], "i_conv": rs["i_conv"], "seed_status": rs["seed_status"],
               "reorth_passes": rs["reorth_passes"], "t_rhs1_ms": t_seed * 1e3, "rhs1_cg_after": rr["iters"][0],
               "rhs2_cg_iters": rr["iters"][1], "rhs2_vs_standard": rr["iters"][1] / std,
               "max_true_relres": max(rr["true_relres"])}
        log(json.dumps(out))
        return out

    ks = [one(k, cfg.past) for k in (10, 20, 50, 100, 200, 250, 0)]
    pasts = [one(cfg.reorth_k, p) for p in (1.0, 1.2, 1.4, 1.6, 2.0)]
    print(json.dumps({"metric": "RHS-1 cost and RHS-2 CG iterations vs reorthogonalisation frequency k and past factor",
                      "config": {"workload": f"Seed-CG fp64 on {'x'.join(map(str, cfg.dims))}, 2 RHS, tol {cfg.tol}",
                                 "kappa": kappa},
                      "standard_cg_iters_rhs2": std, "k_sweep": ks, "past_sweep": pasts}))


def copy_rate():
    """GB/s of a plain 1 GiB device-to-device copy (read + write bytes), timed with events: what HBM
    delivers in practice, beside the 8 TB/s peak."""
    import torch
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del src, dst
    return 2.0 * (1 << 30) / (ms * 1e-3) / 1e9


def roofline_probes():
    """The library's roofline probes on this GPU: copy, FP64 triad and read over 2 GiB buffers (8x the
    256 MB memory-side cache, so HBM serves them), and register-resident FP64 / FP32 matrix-core
    chains; the measured ceilings beside the datasheet's 8 TB/s, 78.6 and 157.3 TFLOP/s."""
    import torch
    from paper_0901_3512_amd import SeedCGError, probe_bandwidth, probe_mfma
    torch.cuda.empty_cache()
    try:
        out = {f"{k}_gbs": probe_bandwidth(k, 1 << 31, 10) for k in ("copy", "triad", "read")}
        out["mfma_f64_tflops"] = probe_mfma("fp64", 20000)
        out["mfma_f32_tflops"] = probe_mfma("fp32", 20000)
    except SeedCGError as e:   # no room for the buffers beside what the run still holds
        log(f"roofline probes skipped: {e}")
        return None
    return out


def with_achievable(roofline, probes):
    """The roofline object with the measured HBM ceiling (the triad probe) and the fraction of it."""
    if roofline.get("unit") == "GB/s" and roofline.get("achieved") and probes:
        roofline["achievable"] = probes["triad_gbs"]
        roofline["frac_achievable"] = roofline["achieved"] / probes["triad_gbs"]
        if roofline.get("combined"):
            roofline["combined_frac_achievable"] = roofline["combined"] / probes["triad_gbs"]
    return roofline


def copy_probe():
    """A plain 1 GiB device copy: the reference for scaling the HBM byte counters."""
    import torch
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def _member_inputs(name):
    from synth.configs import batch_members, make_links, make_sources
    m = {c.name: c for c in batch_members()}[name]
    return make_links(m), make_sources(m)


def bench_batch(args):
    """The batched workload: every member solved by Algorithm 1 + CG inside one seedcg_solve_batch call."""
    import numpy as np
    import torch
    from concurrent.futures import ProcessPoolExecutor
    from paper_0901_3512_amd import SeedCG, SeedCGBatch
    from synth.configs import batch_members, kappa_for

    members = batch_members()[:args.batch_n]
    kappas = [kappa_for(m) for m in members]
    prec = args.prec or members[0].prec
    dev = torch.device("cuda:0")
    t_gen = time.time()
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        inputs = list(ex.map(_member_inputs, [m.name for m in members]))
    log(f"inputs: {len(members)} configurations ({time.time() - t_gen:.1f} s)")
    links = [torch.from_numpy(U).to(dev) for U, _ in inputs]
    B = []
    for m, k, (U, phi), Ud in zip(members, kappas, inputs, links):
        s = SeedCG(Ud, m.dims, k, t_bc=m.t_bc, autotune=False, m_max=2)
        B.append(s.apply_A(torch.from_numpy(phi).to(dev), dagger=True))   # b = A^dag phi (not timed)
        s.close()
    del inputs
    nrhs = B[0].shape[0]
    torch.cuda.synchronize()
    t_c = time.time()
    m0 = members[0]
    batch = SeedCGBatch(links, [m.dims for m in members], kappas, nrhs, t_bc=m0.t_bc, prec=prec, reorth_k=m0.reorth_k,
                        past=m0.past, tol=m0.tol, reliable_every=m0.reliable_every)
    info = batch.info()
    log(f"batch: {info['nclass']} shape classes, m_cap {info['m_cap']}, launch shapes {info['tune']} "
        f"(set-up {time.time() - t_c:.1f} s)")

    def step():
        X, reps = batch.solve(B)
        return X, reps

    for w in range(args.warmup):
        _, reps = step()
        log(f"warmup {w}: m {min(r['m'] for r in reps)}..{max(r['m'] for r in reps)}")
    if args.copy_probe:
        copy_probe()   # marks the start of the timed region in a counter trace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solved, last = 0, None
    for k in range(args.steps):
        X, reps = step()
        last = reps
        solved += sum(1 for r in reps for x in r["true_relres"] if x <= m0.tol)
        log(f"step {k}: max relres {max(max(r['true_relres']) for r in reps):.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the stencil rate, sampled on one more solve (event sampling replaces graph replay by eager launches)
    batch.set_timing(args.sample_every, 16384)
    batch.solve(B)
    torch.cuda.synchronize()
    tm = batch.get_timing()
    batch.set_timing(0, 0)
    hop_ms = tm["ms"] / max(tm["launches"], 1)
    hop_bytes = tm["bytes"] / max(tm["launches"], 1)
    achieved = hop_bytes / (hop_ms * 1e-3) / 1e9 if tm["launches"] else None
    # The classes' launches overlap on their streams, so a sampled launch's event pair also spans
    # what the other classes ran beside it. The algorithmic bytes of every stencil launch of a solve
    # (the same launches as a timed step's, which replays them from graphs) over the timed step's
    # wall time bound the classes' combined stencil rate from below.
    combined = tm["seen_bytes"] / (elapsed / args.steps) / 1e9
    V = sum(int(np.prod(m.dims)) for m in members)
    result = {
        "metric": METRIC, "value": solved / elapsed, "unit": "RHS/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == "fp64" else f"f32+f64({prec})", "data": "synthetic",
        "config": {"workload": f"batched Seed-CG {prec}: {len(members)} configurations of "
                               f"{{8^4, 8^3x16, 12^3x24, 12^4}} ({V} sites), {nrhs} point sources each, tol {m0.tol:g}, "
                               f"k={m0.reorth_k}", "name": "c4", "configurations": len(members), "sites": V,
                   "nrhs": nrhs, "precision": prec},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": measured_traffic(None, None, "hop_", name=f"hop_kernel_batch{len(members)}_{prec}_traffic.txt"),
                     "kernel": "hop kernels of the batch (one launch per shape class, concurrent classes)",
                     "launches_sampled": tm["launches"], "avg_launch_us": hop_ms * 1e3, "avg_launch_bytes": hop_bytes,
                     "solve_launches": tm["seen"], "solve_bytes": tm["seen_bytes"], "combined": combined,
                     "combined_frac": combined / HBM_PEAK_GBS,
                     "combined_note": "algorithmic bytes of every stencil launch of one solve / the timed step's wall "
                                      "time: a lower bound for the concurrent classes' stencil rate together",
                     "traffic_note": "HBM bytes per hop launch averaged over every hop dispatch of one timed solve "
                                     "(rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled); achieved and avg_launch_bytes "
                                     "average the event-sampled launches of one more solve"},
        "cpu_baseline": None,
        "detail": {"classes": info, "m": [r["m"] for r in last], "i_conv": [r["i_conv"] for r in last],
                   "iters": [r["iters"] for r in last], "max_true_relres": max(max(r["true_relres"]) for r in last)},
    }
    batch.close()   # the arena holds most of HBM; the probes need 6 GiB
    probes = roofline_probes()
    with_achievable(result["roofline"], probes)
    result["detail"]["roofline_probes"] = probes
    print(json.dumps(result), flush=True)


def measured_traffic(cfg, tag, kernel=None, name=None):
    """HBM bytes per stencil launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary of this
    workload (and, when given, of this kernel), or None when there is none or the stencil source
    changed since it was taken."""
    from paper_0901_3512_amd.profsummary import source_digest
    name = name or f"hop_kernel_{'x'.join(map(str, cfg.dims))}_{tag}_traffic.txt"
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.startswith("#"))
    # "kernel=<name> dispatches=<n>" (the name holds spaces)
    if kernel is not None and kv.get("kernel", "").rsplit(" dispatches=", 1)[0] != kernel:
        return None
    src = os.path.join(ROOT, "paper_0901_3512_amd", "csrc", "dslash.hip")
    if kv.get("source_sha256_16") != source_digest(src):
        return None
    return float(kv["traffic_bytes_per_launch"])


def cpu_baseline(cfg, U, phi, kappa, rep, n_iter):
    """The FP64 oracle on the host cores, on a bounded sample: n_iter steps of Algorithm 1 on all
    right-hand sides and n_iter CG steps on one, scaled by the GPU run's iteration counts to RHS/s."""
    import numpy as np
    from oracle import seedcg as osc
    from oracle.wilson import WilsonEO, flat, matvec_M, num_threads
    op = WilsonEO(U, cfg.dims, kappa, t_bc=cfg.t_bc)
    mv = matvec_M(op)
    B = flat(op.apply_Adag(phi))
    # (1) Algorithm 1 without reorthogonalisation: cost per Lanczos step with the seeding of every RHS
    t0 = time.perf_counter()
    osc.seed_cg(mv, B, k=0, tol=cfg.tol, m=n_iter)
    t_step = (time.perf_counter() - t0) / n_iter
    # (2) the same reorthogonalised at every step: the extra time per basis vector reorthogonalised against
    t0 = time.perf_counter()
    osc.seed_cg(mv, B, k=1, tol=cfg.tol, m=n_iter)
    t_k1 = time.perf_counter() - t0
    t_vec = max(0.0, t_k1 - t_step * n_iter) / (n_iter * (n_iter + 1) / 2.0)
    # (3) plain CG steps
    t0 = time.perf_counter()
    osc.cg(mv, B[1], None, tol=1e-300, max_iter=n_iter)
    t_cg = (time.perf_counter() - t0) / n_iter
    rs, rr = rep
    m, k = rs["m"], cfg.reorth_k
    reorth_vecs = sum(range(k, m + 1, k)) if k else 0
    t_total = m * t_step + reorth_vecs * t_vec + sum(rr["iters"]) * t_cg
    return {"value": cfg.nrhs / t_total, "unit": "RHS/s", "cores": num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(), "extrapolated": True,
            "sample": f"{n_iter} Algorithm-1 steps on {cfg.nrhs} RHS without and with reorthogonalisation "
                      f"({t_step:.3f} s/step, {t_vec * 1e3:.2f} ms per basis vector reorthogonalised against) and "
                      f"{n_iter} CG steps ({t_cg:.3f} s/step) on {'x'.join(map(str, cfg.dims))}, extrapolated to the "
                      f"GPU run's m={m}, {reorth_vecs} vector reorthogonalisations and {sum(rr['iters'])} CG steps"}


if __name__ == "__main__":
    main()
