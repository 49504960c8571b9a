"""Host-side checks of bench.py: the single-GPU contract and the committed
rocprofv3 traffic summaries it reads its roofline traffic from."""
import glob
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "single-GPU" in capsys.readouterr().err


def test_traffic_summaries_parse():
    files = glob.glob(os.path.join(ROOT, "profiles", "traffic_*.txt"))
    assert files
    for p in files:
        vals = {}
        with open(p) as fh:
            for line in fh:
                if "=" in line and not line.lstrip().startswith("#"):
                    k, v = (t.strip() for t in line.split("=", 1))
                    vals[k] = v
        assert re.fullmatch(r"[0-9a-f]{16}", vals["source_sha256"]), p
        assert float(vals["fetch_bytes_per_launch"]) > 0 and float(vals["write_bytes_per_launch"]) > 0, p
        assert int(vals["launches"]) >= 1, p
        # each summary names the command that produced it, on committed files only
        text = open(p).read()
        assert "rocprofv3" in text and "bench.py" in text and "_work" not in text, p


def test_source_hash_is_stable_and_kernel_specific():
    a = bench.source_hash("row_ProgPhasePropT_f32_N8192")
    assert a == bench.source_hash("row_ProgPropIntensity_f32_N8192")  # one set of row-pass sources
    assert a != bench.source_hash("transpose_8B_N8192")
