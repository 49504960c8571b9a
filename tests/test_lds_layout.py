"""The row FFT's LDS exchange layouts (host logic, no GPU): every plan's
exchanges map the row to distinct slots inside its buffer, and the linear
layouts' one-address-plus-step forms agree with the layout element by
element.  Builds tests/lds_layout_check.cpp with the host compiler."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1301_0514_amd", "csrc")


def test_lds_exchange_layouts(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "lds_layout_check")
    subprocess.run([cxx, "-std=c++17", "-O1", "-I", CSRC, os.path.join(HERE, "lds_layout_check.cpp"), "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-3000:]
    assert r.stdout.strip().endswith("0 failures")
    # the layouts chosen for the rows that needed them: linear 10000 and
    # 20000 buffers within two workgroups per CU (10000) and the LDS (20000)
    assert "ok L=10000 V=1 eb=8 buffer=10100" in r.stdout
    assert "ok L=20000 V=1 eb=8 buffer=20100" in r.stdout
