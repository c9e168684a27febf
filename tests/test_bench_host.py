"""Host-side parts of the benchmark: the one-GPU restriction, the gating of
the committed HBM counters by the kernel sources, the CPU-baseline leg and
the algorithmic-work constants.  No GPU needed."""
import json
import os
import subprocess
import sys

import numpy as np

import bench
import saa_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_traffic_only_for_the_sources_it_was_measured_on():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        data = json.load(fh)
    for key, ent in data.items():
        assert bench._traffic(key, ent["source_hash"]) == ent["bytes_per_launch"]
        assert bench._traffic(key, "0" * 16) is None
        assert os.path.exists(os.path.join(ROOT, ent["summary"]))
    assert bench._traffic("no such kernel", "0" * 16) is None


def test_cpu_baseline_record():
    import paper_2305_20053_amd as saa
    prob = saa.Problem(n=8, kl_per_dim=4)
    xi = si.kl_coefficients(2421, 64, prob.kl_per_dim)
    rec = bench.cpu_baseline(prob, xi, si.control(2422), seconds_target=0.5)
    assert set(rec) == {"value", "unit", "cores", "kind", "sample", "host_cpu_count", "usable_cores"}
    assert rec["kind"] == "oracle" and rec["unit"] == "samples/s"
    assert 1 <= rec["cores"] <= 16 and rec["value"] > 0
    assert rec["cores"] == min(16, rec["usable_cores"]) and rec["host_cpu_count"] == os.cpu_count()
    assert "n=8" in rec["sample"]


def test_surrogate_flop_count():
    # 1.068 MFLOP per sample: forward through 125 -> 256^4 -> 200 and the
    # reverse pass down to the 25 controls, two flops per multiply-add
    fwd = [(125, 256), (256, 256), (256, 256), (256, 256), (256, 200)]
    rev = [(200, 256), (256, 256), (256, 256), (256, 256), (256, 25)]
    assert bench.MRDINO_FLOP_PER_SAMPLE == sum(2 * a * b for a, b in fwd + rev) == 1068032
    assert np.isclose(bench.MRDINO_FLOP_PER_SAMPLE * 65536 / 1e9, 70.0, atol=0.01)
