"""The benchmark's synthetic workloads as documented: sizes, q-rounding (multiples of 2^-15, exact in FP32),
positions inside the box, periodic directions and referring transforms."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

Q = 2.0 ** -15


def _q_rounded(x):
    return np.array_equal(x / Q, np.round(x / Q))


def test_channel_workload():
    wl = bench.workload("channel")
    # FCC 238 x 119 x 59 unit cells of 4 sites in the 400 x 200 x 100 channel
    assert wl.n == 4 * 238 * 119 * 59 == 6683992
    assert wl.mesh.n_cells == 4312968
    assert _q_rounded(wl.x)
    assert np.all(wl.x >= wl.box_lo) and np.all(wl.x < wl.box_hi)
    assert wl.periodic_axes == (0, 2) and wl.rotations is None
    per = np.asarray(wl.lattice)
    assert per.shape == (2, 3) and np.allclose(per, [[400.0, 0, 0], [0, 0, 100.0]])
    rho = wl.n / np.prod(wl.box_hi - wl.box_lo)
    assert abs(rho - 0.8356) < 1e-3
    assert np.all(wl.species == 0) and wl.rcut == 2.5


def test_wedge_workload():
    wl = bench.workload("wedge")
    assert wl.n == 371896 and wl.mesh.n_cells == 373500
    assert _q_rounded(wl.x)
    w = wl.mesh.wedge
    assert w["n_sectors"] == 12 and abs(w["theta"] - np.pi / 6) < 1e-15
    r = np.hypot(wl.x[:, 0], wl.x[:, 1])
    phi = np.arctan2(wl.x[:, 1], wl.x[:, 0])
    assert r.min() > 100.0 and r.max() < 200.0
    assert phi.min() > 0.0 and phi.max() < np.pi / 6
    assert np.all((wl.x[:, 2] >= 0) & (wl.x[:, 2] < 60.0))
    R = np.asarray(wl.rotations)
    # one rotation by 30 degrees about z (the coupled sides) and the z translation (identity rotation)
    assert R.shape[0] == 2 and np.allclose(R[0] @ R[0].T, np.eye(3)) and abs(np.linalg.det(R[0]) - 1) < 1e-12
    assert abs(np.arctan2(R[0][1, 0], R[0][0, 0]) - np.pi / 6) < 1e-12
    assert np.allclose(R[1], np.eye(3))
