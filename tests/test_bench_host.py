"""CPU tests of the benchmark's host side: the one-GPU guard and the reading of the committed counter
summaries (used only while the kernel sources hash to the digest they were taken on)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "error" in out


def test_counter_summaries_follow_the_source_digest(monkeypatch):
    digest = bench.kernel_digest()
    assert len(digest) == 16
    traffic = {k: bench.measured_traffic(k, "channel") for k in ("pair_fwd", "pair_adj")}
    valu = {k: bench.measured_valu_issue(k, "channel") for k in ("pair_fwd", "pair_adj")}
    with open(os.path.join(ROOT, "profiles", "traffic_channel.txt")) as fh:
        committed = [line.split()[1] for line in fh if line.startswith("sources_sha256:")]
    assert len(committed) == 1
    if committed[0] == digest:  # summaries taken on these sources: plausible values
        assert all(v is not None and 1e8 < v < 1e11 for v in traffic.values()), traffic
        assert all(v is not None and 0.0 < v <= 1.0 for v in valu.values()), valu
    # any other source digest makes both readers return None
    monkeypatch.setattr(bench, "kernel_digest", lambda: "0" * 16)
    assert bench.measured_traffic("pair_adj", "channel") is None
    assert bench.measured_valu_issue("pair_adj", "channel") is None
    assert bench.measured_traffic("pair_adj", "no_such_workload") is None
