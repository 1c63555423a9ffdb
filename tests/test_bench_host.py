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


def test_moving_sets_stay_in_the_mesh_on_the_grid():
    """The benchmark's per-step position sets: set 0 is the workload, later sets move by k delta (about
    0.005 sigma per step and coordinate), stay on the 2^-15 position grid, inside the box, wrapped on the
    periodic axes and reflected at the walls."""
    import numpy as np

    from paper_cs_0702131_amd import workloads as W
    for wl in (W.config1(), W.small_random(N=300, periodic_axes=(0, 2), seed=3)):
        sets = bench.moving_sets(wl, 6)
        assert len(sets) == 6 and sets[0] is wl.x
        lo, hi = wl.mesh.lo, wl.mesh.hi
        for k, x in enumerate(sets[1:], start=1):
            assert np.all(x >= lo) and np.all(x <= hi)
            assert np.array_equal(W.qround(x), x)
            d = x - wl.x
            for a in wl.periodic_axes:
                L = hi[a] - lo[a]
                d[:, a] -= L * np.round(d[:, a] / L)
            step = np.sqrt((d ** 2).mean())
            assert 0.5 * 0.005 * k < step < 1.5 * 0.005 * k, (k, step)
        for a in wl.periodic_axes:
            assert all(np.all(x[:, a] < hi[a]) for x in sets)
