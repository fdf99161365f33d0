"""The benchmark's command-line contract that holds without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_table_is_well_formed():
    """profiles/traffic.json: per step-kernel instantiation and workload, the
    scaled FETCH_SIZE and WRITE_SIZE bytes per launch, their sum, and the hash
    of the kernel sources they were taken with (bench.py reports them only
    while that hash matches)."""
    import json
    data = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert data, "no byte counters recorded"
    for key, ent in data.items():
        assert key.startswith("k_em_step<") and "@" in key, key
        assert ent["bytes_per_launch"] == ent["fetch_bytes"] + ent["write_bytes"]
        assert len(ent["kernels_sha"]) == 16
        assert os.path.exists(os.path.join(ROOT, ent["source"])), ent["source"]
