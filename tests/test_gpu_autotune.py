"""The autotuner's persisted choice (DPD_TUNE_CACHE): written after timing,
then taken by later calls for the same class of system, in this process and
in another, without timing; every variant still gives the same bits (the
variant tests in test_gpu_parity.py cover the whole table)."""
import json
import os
import subprocess
import sys
import time

import pytest

from paper_1804_06205_amd import dpd
from paper_1804_06205_amd import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dpd.lib()


_CHILD = """
import sys
sys.path.insert(0, {root!r})
from paper_1804_06205_amd import dpd, workloads as W
w = W.melt(12.0, seed=53)
with dpd.System.from_workload(w) as g:
    g.step(2)
    v, ms = g.autotune(2)
print(v, repr(ms))
"""


def test_autotune_cache_is_written_and_reused(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("DPD_TUNE_CACHE", str(path))
    w = W.melt(12.0, seed=52)
    with dpd.System.from_workload(w) as g:
        g.step(2)
        v, ms = g.autotune(2)
    entries = json.loads(path.read_text())
    assert len(entries) == 1
    (key, ent), = entries.items()
    assert ent["variant"] == v and ent["ms"] == ms and "mixed" in key
    # Same class in this process: the stored choice, to the bit.
    with dpd.System.from_workload(W.melt(12.0, seed=54)) as g:
        g.step(1)
        t0 = time.perf_counter()
        v2, ms2 = g.autotune(5)
        dt = time.perf_counter() - t0
    assert (v2, ms2) == (v, ms)
    print(f"cached autotune call {dt * 1e3:.2f} ms", flush=True)
    # Another process, another system of the class.
    env = dict(os.environ, DPD_TUNE_CACHE=str(path))
    out = subprocess.run([sys.executable, "-c", _CHILD.format(root=ROOT)], env=env,
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    v3, ms3 = out.stdout.split()
    assert int(v3) == v and float(ms3) == ms
    # An entry the library did not time is taken as it stands: nothing is timed.
    other = (v + 1) % len(dpd.variants())
    path.write_text(json.dumps({key: {"variant": other, "ms": 123.0}}))
    with dpd.System.from_workload(w) as g:
        g.step(1)
        assert g.autotune(2) == (other, 123.0)
    # Another class (a different box size) is timed and added.
    with dpd.System.from_workload(W.melt(8.0, seed=55)) as g:
        g.step(1)
        v4, ms4 = g.autotune(2)
    entries = json.loads(path.read_text())
    assert len(entries) == 2 and entries[key]["ms"] == 123.0
