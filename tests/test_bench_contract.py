"""Host-side parts of the benchmark contract (no GPU): the one-GPU refusal and the traffic figure's
source check."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_traffic_is_reported_only_for_the_current_stencil_source():
    sys.path.insert(0, ROOT)
    import bench
    from synth.configs import CONFIGS
    from paper_0901_3512_amd.profsummary import source_digest
    cfg = CONFIGS["c2"]
    path = os.path.join(ROOT, "profiles", "hop_kernel_16x16x16x32_fp64_traffic.txt")
    kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.startswith("#"))
    src = os.path.join(ROOT, "paper_0901_3512_amd", "csrc", "dslash.hip")
    current = kv["source_sha256_16"] == source_digest(src)
    t = bench.measured_traffic(cfg, "fp64")
    assert (t == float(kv["traffic_bytes_per_launch"])) if current else (t is None)


def test_dominant_kind_names_the_rocprof_kernel_and_traffic_needs_that_kernel():
    sys.path.insert(0, ROOT)
    import bench
    from synth.configs import CONFIGS
    kinds = [dict(fmt=3, nvec=1, fused=0, tps=8, vb=1, launches=100, ms=5.0, bytes=8e9),
             dict(fmt=4, nvec=11, fused=1, tps=8, vb=2, launches=10, ms=9.0, bytes=9e9)]
    d = bench.dominant_kind(kinds)
    assert d["nvec"] == 11 and abs(d["avg_us"] - 900.0) < 1e-9 and abs(d["gbs"] - 1000.0) < 1e-9
    assert bench.kind_kernel(d) == "scg::hop_split_kernel<float, scg::su3rows<float>, 2, true>"
    assert bench.kind_tag(d) == "fp32_split_vb2_cgu"
    assert bench.kind_kernel(dict(fmt=0, nvec=1, fused=0, tps=10, vb=1)) == "scg::hop_quad_kernel<double, double, false>"
    assert bench.kind_kernel(dict(fmt=3, nvec=1, fused=0, tps=12, vb=1)) == "scg::hop_quad_nt_kernel<double, scg::su3rows<double>, false>"
    assert bench.kind_tag(dict(fmt=3, nvec=1, fused=0, tps=12, vb=1)) == "fp64_quadnt_vb1"
    # a traffic summary of another kernel is never used for this one
    assert bench.measured_traffic(CONFIGS["c2"], "fp64", "scg::some_other_kernel") is None


def test_headline_traffic_summary_is_found_for_its_own_kernel():
    """The committed 24^3 x 48 summaries of the one-vector FP64 launches (non-temporal quad split) and
    of the 23-vector FP32 ones name their kernel on a line that also carries the dispatch count; the
    lookup takes the name alone and needs the current source."""
    sys.path.insert(0, ROOT)
    import bench
    from synth.configs import CONFIGS
    from paper_0901_3512_amd.profsummary import source_digest
    for k in (dict(fmt=3, nvec=1, fused=0, tps=12, vb=1), dict(fmt=4, nvec=23, fused=0, tps=11, vb=1)):
        path = os.path.join(ROOT, "profiles", f"hop_kernel_24x24x24x48_{bench.kind_tag(k)}_traffic.txt")
        kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.startswith("#"))
        assert kv["kernel"].rsplit(" dispatches=", 1)[0] == bench.kind_kernel(k)
        current = kv["source_sha256_16"] == source_digest(os.path.join(ROOT, "paper_0901_3512_amd", "csrc", "dslash.hip"))
        t = bench.measured_traffic(CONFIGS["c3t"], bench.kind_tag(k), bench.kind_kernel(k))
        assert (t == float(kv["traffic_bytes_per_launch"])) if current else (t is None)
        assert bench.measured_traffic(CONFIGS["c3t"], bench.kind_tag(k), "scg::hop_split_kernel<double, double, 1, false>") is None
