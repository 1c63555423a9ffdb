"""GPU test of aica_forces_noalloc (every buffer of the call in the library's fixed scratch array) against
aica_forces on the same binned positions: forces, U, W and the pair count must agree bit for bit, on calls in
a row whose inputs shrink, so that records left in the array by a larger call cannot leak into a smaller one."""
import sys

import numpy as np
import pytest

from paper_cs_0702131_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_cs_0702131_amd as pkg
    pkg.lib()
    return pkg


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _two_species(wl, frac, seed):
    rng = np.random.default_rng(seed)
    wl.species = (rng.random(wl.n) < frac).astype(np.int32)
    wl.eps = np.array([1.0, 0.6])
    wl.sigma = np.array([1.0, 0.85])
    return wl


def _workloads():
    big = _two_species(W.fcc_cube(13.44, 5, 8, jitter=0.05, seed=31, name="fcc2048_mesh5"), 0.4, 32)
    mid = W.config1(seed=33)
    small = W.small_random(n_mesh=(4, 3, 5), L=(8.5, 7.0, 9.0), N=300, periodic_axes=(0, 2), seed=34,
                           species_frac=0.6)
    wedge = W.wedge(seed=35, nr=6, nphi=5, nz=4)
    return [big, mid, small, wedge, mid]


def _compare(A, wl, precision, compensated=True):
    import torch
    dt = torch.float64 if precision == "fp64" else torch.float32
    d = A.DIL(wl.mesh, wl.rcut)
    x = torch.tensor(wl.x, dtype=dt, device="cuda")
    sp = torch.tensor(wl.species, dtype=torch.int32, device="cuda")
    A.aica_bin(d, x)
    F0, uw0, np0 = A.aica_forces(d, x, sp, wl.eps, wl.sigma, precision=precision, compensated=compensated)
    n = wl.n
    out = (torch.full((n, 3), float("nan"), dtype=dt, device="cuda"),
           torch.full((2,), float("nan"), dtype=torch.float64, device="cuda"),
           torch.full((1,), -1, dtype=torch.int64, device="cuda"))
    F1, uw1, np1 = A.aica_forces_noalloc(d, x, sp, wl.eps, wl.sigma, precision=precision,
                                         compensated=compensated, out=out)
    torch.cuda.synchronize()
    assert F1.data_ptr() == out[0].data_ptr()
    assert int(np1.cpu()[0]) == int(np0.cpu()[0]) > 0
    assert torch.equal(F1, F0), (wl.name, precision, (F1 - F0).abs().max().item())
    assert torch.equal(uw1, uw0), (wl.name, precision, uw1.cpu().numpy(), uw0.cpu().numpy())
    return d, x


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_matches_forces_on_shrinking_calls(A, precision):
    wls = _workloads()
    assert [w.n for w in wls[:3]] == sorted((w.n for w in wls[:3]), reverse=True)
    for k, wl in enumerate(wls):
        _note(f"no-alloc call {k}: {wl.name} n={wl.n} {precision}")
        _compare(A, wl, precision)


def test_noalloc_uncompensated_and_repeat(A):
    import torch
    wl = W.config1(seed=36)
    _note(f"no-alloc uncompensated: {wl.name} n={wl.n}")
    d, x = _compare(A, wl, "fp32", compensated=False)
    # the same step twice through the fixed array: identical results
    a = A.aica_forces_noalloc(d, x, None, wl.eps, wl.sigma, precision="fp32")
    b = A.aica_forces_noalloc(d, x, None, wl.eps, wl.sigma, precision="fp32")
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        assert torch.equal(u, v)


def test_noalloc_rejects_a_step_beyond_the_array(A):
    """1.5M molecules in FP64 need 144 MB for positions and own records alone (the array holds 128 MiB):
    the call fails with AICA_E_INVAL before launching anything, and a later small call still works."""
    import torch
    L, n = 80.0, 1_500_000
    nodes = W.uniform_nodes(L, 16)
    mesh = W.hex_mesh(nodes, nodes, nodes, periodic_axes=(0, 1, 2))
    x = W.qround(np.random.default_rng(37).uniform(0.0, L, size=(n, 3)))
    x = np.where(x >= L, x - L, x)
    _note(f"no-alloc rejection: n={n} fp64")
    d = A.DIL(mesh, 2.5)
    xt = torch.tensor(x, dtype=torch.float64, device="cuda")
    A.aica_bin(d, xt)
    with pytest.raises(Exception, match="scratch"):
        A.aica_forces_noalloc(d, xt, None, precision="fp64")
    del xt, d
    _compare(A, W.config1(seed=38), "fp64")
