"""bench.py's host logic that needs no GPU: more than one GPU is refused with
a message (this library measures and runs one GPU), and the counter-based
traffic figure is tied to the kernel source it was measured on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bench_refuses_a_multi_rank_launch():
    env = dict(os.environ, WORLD_SIZE="2")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")], capture_output=True, text=True,
                       timeout=120, env=env)
    assert r.returncode == 2 and "one GPU" in r.stderr


def _bench_module():
    import importlib.util

    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_is_reported_only_for_the_profiled_kernels(tmp_path):
    """The roofline's traffic comes from the committed counter summary only while the kernel
    source it was measured on is unchanged: a changed source gives null."""
    import json
    import shutil

    import hashlib

    bench = _bench_module()
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    src_path = os.path.join(ROOT, "paper_2502_03749_amd", "csrc", "pins_kernels.hip")
    current = rec["kernels_sha256"] == hashlib.sha256(open(src_path, "rb").read()).hexdigest()
    assert bench._traffic("pcg") == (rec["per_launch_bytes"]["pcg"] if current else None)
    assert bench._traffic("no_such_kernel") is None
    # the same record beside an edited kernel source
    (tmp_path / "profiles").mkdir()
    shutil.copy(os.path.join(ROOT, "profiles", "traffic.json"), tmp_path / "profiles" / "traffic.json")
    csrc = tmp_path / "paper_2502_03749_amd" / "csrc"
    csrc.mkdir(parents=True)
    src = open(os.path.join(ROOT, "paper_2502_03749_amd", "csrc", "pins_kernels.hip")).read()
    (csrc / "pins_kernels.hip").write_text(src + "\n// edited\n")
    bench.ROOT = str(tmp_path)
    assert bench._traffic("pcg") is None
