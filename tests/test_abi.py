"""The C ABI library loads and exports every symbol include/dpd.h declares.
No compute calls: these run without a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1804_06205_amd import dpd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpd_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_step_path_calls():
    names = _declared()
    for must in ("dpd_create", "dpd_set_params", "dpd_add_bonds", "dpd_step",
                 "dpd_observables", "dpd_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = dpd.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", dpd.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (dpd_[a-z_0-9]+)$", out, flags=re.M))
    for name in _declared():
        assert name in exported, name
        assert getattr(lib, name) is not None
    # The binding wraps exactly the declared calls.
    assert sorted(dpd.SIGNATURES) == _declared()


def test_exports_are_plain_c():
    # No C++ or torch types cross the boundary: every dpd_ symbol is unmangled.
    out = subprocess.run(["nm", "-D", "--defined-only", dpd.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for line in out.splitlines():
        if "dpd_" in line and " T " in line:
            assert not line.split()[-1].startswith("_Z"), line


def test_version_and_structs():
    assert dpd.lib().dpd_version() == 1
    # dpd_obs: int64 step, 8 doubles (time .. pressure), 3 momentum, int64 npairs.
    assert ctypes.sizeof(dpd.Obs) == 8 + 8 * 8 + 3 * 8 + 8
    assert ctypes.sizeof(dpd.KernelTimes) == 6 * 8


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_1804_06205_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text and "dpd_oracle" not in text, f


def test_create_without_gpu_fails_cleanly():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    import numpy as np
    with pytest.raises(dpd.DPDError) as e:
        dpd.System([5.0] * 3, np.random.rand(10, 3) * 5, np.zeros((10, 3)))
    assert e.value.code == dpd.EDEVICE
    assert dpd.last_error()


@pytest.mark.parametrize("n", [0, 1])
def test_create_rejects_fewer_than_two_particles(n):
    # Argument checks come before any device call, so this runs without a GPU.
    import numpy as np
    with pytest.raises(dpd.DPDError) as e:
        dpd.System([5.0] * 3, np.random.rand(n, 3) * 5, np.zeros((n, 3)))
    assert e.value.code == dpd.EINVAL
    assert dpd.last_error()
