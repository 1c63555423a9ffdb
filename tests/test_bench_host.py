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
    ctr = {k: bench.measured_counters(k, "channel") for k in ("pair_fwd", "pair_adj")}
    with open(os.path.join(ROOT, "profiles", bench.COUNTERS_FILE.format(workload="channel"))) as fh:
        committed = [line.split()[1] for line in fh if line.startswith("sources_sha256:")]
    assert len(committed) == 1
    if committed[0] == digest:  # summaries taken on these sources: plausible values
        for c in ctr.values():
            assert 1e8 < c["traffic"] < 1e11 and 0.0 < c["valu_issue_frac"] <= 1.0, c
            assert 1e9 < c["executed_flop"] < 1e13, c
    # any other source digest makes the reader return nothing
    monkeypatch.setattr(bench, "kernel_digest", lambda: "0" * 16)
    assert bench.measured_counters("pair_adj", "channel") == {}
    assert bench.measured_counters("pair_adj", "no_such_workload") == {}


def test_pmc_summary_lines(tmp_path):
    """The counter summariser on a hand-written rocprofv3 CSV: means over dispatches, the issue fraction
    against one instruction per CU per cycle, executed FLOPs as 64 lanes x the per-instruction counters, and
    the traffic line with the copy calibration's scale (512 MiB copied, counters reading half of it)."""
    head = '"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value","Start_Timestamp","End_Timestamp"\n'
    k = bench.PAIR_KERNELS["pair_adj"]
    rows = []
    for disp, (valu, f32) in enumerate([(6.0e8, 1.0e8), (6.4e8, 1.2e8)], start=1):
        t0, t1 = 1000, 1000 + 2_000_000  # 2 ms
        for c, v in (("SQ_INSTS_VALU", valu), ("SQ_INSTS_VALU_FLOPS_FP32", f32), ("SQ_INSTS_VALU_FLOPS_FP32_TRANS", 1e6),
                     ("SQ_INSTS_VALU_FLOPS_FP64", 2e6), ("SQ_INSTS_VALU_FLOPS_FP64_TRANS", 0.0),
                     ("FETCH_SIZE", 1000.0), ("WRITE_SIZE", 3000.0)):
            rows.append(f'{disp},"void (anonymous namespace)::{k}(float const*)","{c}",{v},{t0},{t1}\n')
    p = tmp_path / "run.csv"
    p.write_text(head + "".join(rows))
    cf = tmp_path / "cf.csv"
    cf.write_text(head + '1,"__amd_rocclr_copyBuffer","FETCH_SIZE",262144.0,0,10\n')
    cw = tmp_path / "cw.csv"
    cw.write_text(head + '1,"__amd_rocclr_copyBuffer","WRITE_SIZE",524288.0,0,10\n')
    out = bench.pmc_summary([str(p)], str(cf), str(cw), 512).splitlines()
    line = {f.split()[0] + f.split()[1]: f.split()[2:] for f in out if not f.startswith("#") and len(f.split()) > 2}
    assert abs(float(line["issue:pair_adj"][0]) - 6.2e8 / 2e-3 / (256 * 2.4e9)) < 1e-4
    assert abs(float(line["flops:pair_adj"][0]) - 64 * (1.1e8 + 1e6 + 2e6)) < 1e3
    assert [float(v) for v in line["traffic:pair_adj"]] == [1000.0, 2.0, 3000.0, 1.0]
    assert out[-1] == f"sources_sha256: {bench.kernel_digest()}"


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
