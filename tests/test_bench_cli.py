"""bench.py's contract parts that need no GPU: more than one GPU is refused
with a message, and the committed rocprofv3 summary it reads the traffic
from parses to the fields it uses."""
import importlib.util
import json
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_profile_summary_has_the_fields_bench_reads():
    f = os.path.join(ROOT, "profiles", "k_align_cfg2.md")
    m = re.search(r"```json\n(.*?)\n```", open(f).read(), re.S)
    d = json.loads(m.group(1))
    for k in ("workload", "kernel_src_sha256_16", "lanes", "traffic_bytes_per_launch", "avg_ns",
              "fetch_scale", "write_scale"):
        assert k in d
    assert d["workload"] == "cfg2" and d["traffic_bytes_per_launch"] > 0
    # the calibration copy moves 1 GiB: the scale factors are what the counters
    # read for it (FETCH_SIZE counts half of a copy's reads on this chip)
    assert 0.5 < d["fetch_scale"] < 4 and 0.5 < d["write_scale"] < 4


def test_roofline_bytes_per_unit_are_the_documented_ones():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    assert (b.B_ENTRY, b.B_CHUNK, b.B_CROSS) == (32, 16, 24)
    assert b.HBM_PEAK_GBS == 8000.0
