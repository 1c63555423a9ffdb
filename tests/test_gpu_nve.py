"""Nanochannel with posts (six cylinders, reflecting walls): 100 velocity-Verlet steps with FP32 pair
arithmetic against the same run in FP64, from identical initial state.

The energy is E = KE + U - npairs u(rc) (the truncated potential shifted to zero at rc).  Molecules
crossing rc receive the force jump F(rc) in both runs, so E is compared between the runs (its drift
and its largest excursion per molecule), not against zero; positions are compared directly.  The
FP64 forces at step 0 are checked against the oracle on sampled rows."""
import numpy as np
import pytest

from paper_cs_0702131_amd import workloads as W

pytestmark = pytest.mark.gpu

U_RC = 4.0 * (2.5 ** -12 - 2.5 ** -6)


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_cs_0702131_amd as pkg
    pkg.lib()
    return pkg


def run_nve(A, d, wl, precision, steps=100, dt=0.005):
    """Velocity Verlet on the device; positions are kept multiples of q after every move."""
    import torch
    dev = "cuda"
    x = torch.tensor(wl.x, dtype=torch.float64, device=dev)
    v = torch.tensor(wl.extra["v"], dtype=torch.float64, device=dev)
    posts = wl.extra["posts"]
    R = wl.extra["post_r"] + 1e-4  # reflect just outside the deleted cells (q-rounding stays outside)
    L = [float(b) for b in wl.box_hi]

    routes = []

    def forces(x):
        A.aica_bin(d, x)
        inf = d.info()
        routes.append((inf["located_ball"], inf["located_record"], inf["located_search"]))
        F, uw, npairs = A.aica_forces(d, x, None, wl.eps, wl.sigma, precision=precision)
        return F.double(), float(uw[0].item()), int(npairs.item())

    F, U, npairs = forces(x)
    E = [0.5 * float((v * v).sum().item()) + U - npairs * U_RC]
    for _ in range(steps):
        v = v + 0.5 * dt * F
        x = x + dt * v
        for lim, sgn in ((0.0, 1.0), (L[1], -1.0)):  # walls at y = 0 and y = Ly
            m = sgn * (x[:, 1] - lim) < 0
            x[m, 1] = 2 * lim - x[m, 1]
            v[m, 1] = -v[m, 1]
        for px, py in posts:
            dx, dy = x[:, 0] - px, x[:, 1] - py
            r = torch.sqrt(dx * dx + dy * dy)
            m = r < R
            if bool(m.any()):
                nx, ny = dx[m] / r[m], dy[m] / r[m]
                rn = 2 * R - r[m]
                x[m, 0] = px + nx * rn
                x[m, 1] = py + ny * rn
                vn = v[m, 0] * nx + v[m, 1] * ny
                v[m, 0] = v[m, 0] - 2 * vn * nx
                v[m, 1] = v[m, 1] - 2 * vn * ny
        x = torch.round(x / W.Q) * W.Q
        for ax in (0, 2):
            x[:, ax] = torch.remainder(x[:, ax], L[ax])
            x[:, ax] = torch.where(x[:, ax] >= L[ax], x[:, ax] - L[ax], x[:, ax])
        F, U, npairs = forces(x)
        v = v + 0.5 * dt * F
        E.append(0.5 * float((v * v).sum().item()) + U - npairs * U_RC)
    r = np.array(routes[2:], dtype=np.float64)  # after the first two binnings (no history, then no balls)
    print(f"{precision}: molecules per binning located by ball / record / search: "
          f"{r[:, 0].mean():.0f} / {r[:, 1].mean():.0f} / {r[:, 2].mean():.0f}", flush=True)
    return x.cpu().numpy(), np.array(E)


def test_posts_nve_fp32_vs_fp64(A, oracle):
    import torch
    wl = W.config3()
    n = wl.n
    print(f"case {wl.name}: {wl.mesh.n_cells} cells, {n} molecules", flush=True)
    d = A.DIL(wl.mesh, wl.rcut)
    # step-0 forces against the oracle on sampled rows
    rows = np.random.default_rng(31).choice(n, 256, replace=False)
    Fr, Ur, Wr, cnt = oracle.forces_rows(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, rows)
    rms = np.sqrt((Fr ** 2).sum(1).mean())
    x = torch.tensor(wl.x, dtype=torch.float64, device="cuda")
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        A.aica_bin(d, x)
        F, uw, npairs = A.aica_forces(d, x, None, wl.eps, wl.sigma, precision=prec)
        e = np.sqrt(((F.double().cpu().numpy()[rows] - Fr) ** 2).sum(1)).max() / rms
        print(f"step 0 {prec}: e_F {e:.2e} on {len(rows)} rows", flush=True)
        assert e < tol
    x64, E64 = run_nve(A, d, wl, "fp64")
    x32, E32 = run_nve(A, d, wl, "fp32")
    drift64, drift32 = (E64[-1] - E64[0]) / n, (E32[-1] - E32[0]) / n
    dev64, dev32 = np.abs(E64 - E64[0]).max() / n, np.abs(E32 - E32[0]).max() / n
    dx = x32 - x64
    for ax in (0, 2):
        dx[:, ax] -= wl.box_hi[ax] * np.round(dx[:, ax] / wl.box_hi[ax])
    dxmax = np.abs(dx).max()
    print(f"drift/N fp64 {drift64:.3e} fp32 {drift32:.3e}; max |E-E0|/N fp64 {dev64:.3e} fp32 {dev32:.3e}; "
          f"max |x32-x64| {dxmax:.3e}", flush=True)
    # measured on MI355X: drift/N -7.38e-5 (both), max |E - E0|/N 3.63e-4 (both), max |x32 - x64| 3.1e-4
    assert abs(E32[0] - E64[0]) / n < 1e-6
    assert abs(drift32 - drift64) < 1e-5
    assert abs(dev32 - dev64) < 1e-5
    assert dev64 < 1e-3
    assert dxmax < 1e-3
