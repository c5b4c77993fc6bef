"""Benchmark command line checks that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert "{" not in r.stdout  # no benchmark line


def test_committed_counter_summary_is_consistent():
    """The committed byte-counter summary the benchmark scales its traffic figure from: taken
    on the current kernel sources (else the benchmark reports traffic as null, and this
    check is skipped), per-kernel read and write bytes present, and a fan-out total between
    the 44-byte algorithmic model and twice it per edge event."""
    import json

    import pytest
    sys.path.insert(0, ROOT)
    import bench
    with open(bench.COUNTERS_JSON) as f:
        c = json.load(f)
    if c.get("kernel_source_hash") != bench.kernel_source_hash():
        pytest.skip("kernel sources changed since the counters were taken (traffic is reported as null)")
    per_bin = 0.0
    for k in bench.FANIN_KERNELS:
        rw = c["bytes_per_bin"][k]
        assert rw["read"] > 0 and rw["write"] > 0
        per_bin += rw["read"] + rw["write"]
    per_event = per_bin / c["edge_events_per_bin"]
    assert bench.BYTES_PER_EVENT <= per_event <= 2 * bench.BYTES_PER_EVENT
    txt = open(os.path.join(ROOT, "profiles", "fanin_share6.1M_15hz.txt")).read()
    assert "rocprofv3 --kernel-trace --stats" in txt and "--pmc FETCH_SIZE" in txt and "--pmc WRITE_SIZE" in txt
