"""bench.py's host-side contract, on the CPU: the one-GPU refusal, and that the
measured traffic and VALU figures are taken from a committed profile summary only
while its kernel sources and brick match."""
import hashlib
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_profile_figures_need_matching_sources_and_brick(tmp_path):
    b = _bench()
    h = hashlib.sha256()
    for f in b.KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    good = tmp_path / "good.md"
    good.write_text(f"text\n    traffic_bytes_per_launch=123456 variant=1 sources_sha256={h.hexdigest()}\n")
    stale = tmp_path / "stale.md"
    stale.write_text("    traffic_bytes_per_launch=123456 variant=1 sources_sha256=" + "0" * 64 + "\n")
    assert b._profiled(str(good), "traffic_bytes_per_launch", 1) == 123456.0
    assert b._profiled(str(good), "traffic_bytes_per_launch", 2) is None      # other brick
    assert b._profiled(str(stale), "traffic_bytes_per_launch", 1) is None     # other sources
    assert b._profiled(str(tmp_path / "missing.md"), "traffic_bytes_per_launch", 1) is None
    assert b._profiled(str(good), "valu_insts_per_particle", 1) is None       # other figure
