"""The benchmark's contract without a GPU: one GPU only, the counter summary it reads is
present, covers every workload line and was taken on the current kernel sources."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_traffic_summary_matches_the_kernel_sources():
    b = _bench()
    for f in b.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_2412_09051_amd", "csrc", f)), f
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    h = b.kernel_source_hash()
    for key in ("tgv_f64", "tgv_f32", "tgv45_f64", "tgv45_f32", "ogrid_f64", "ogrid_f32", "ogrid19_f64", "ogrid19_f32",
                "c1r_f64", "c1r_f32", "c4_f32", "c4pr_f32", "c4paper_f32",
                "c1rq19_f64", "c1rq19_f32"):
        e = d[key]
        assert e["kernel_source_hash"] == h, (key, "counters taken on other kernel sources: re-profile")
        assert e["bytes_per_launch"] == e["read_bytes"] + e["write_bytes"] > 0
        assert b.traffic_from_profiles(key) == e["bytes_per_launch"]
