"""GPU parity of the hand-written adjoint: against the oracle's analytic gradient,
FP64 central finite differences, torch.autograd.gradcheck, and identities.  Bars: FP64 1e-12; FP32
1e-6 (the pair terms are formed and summed per molecule in FP64 in both precisions, so only the
roundings of the partial sums and of the result to FP32 remain)."""
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


def gpu_adjoint(A, wl, G, gamma, precision, dil=None):
    import torch
    d = dil or A.DIL(wl.mesh, wl.rcut)
    dt = torch.float64 if precision == "fp64" else torch.float32
    x = torch.tensor(wl.x, dtype=dt, device="cuda")
    sp = torch.tensor(wl.species, dtype=torch.int32, device="cuda")
    A.aica_bin(d, x)
    Gt = torch.tensor(G, dtype=dt, device="cuda")
    gx, ge, gs = A.aica_forces_adjoint(d, x, Gt, gamma, sp, wl.eps, wl.sigma, precision=precision)
    F, uw, npairs = A.aica_forces(d, x, sp, wl.eps, wl.sigma, precision=precision)
    torch.cuda.synchronize()
    L = float((G * F.double().cpu().numpy()).sum() + gamma * uw[0].item())
    return gx.double().cpu().numpy(), ge.cpu().numpy(), gs.cpu().numpy(), L


def rel_max(a, b):
    return np.abs(a - b).max() / np.sqrt((b ** 2).mean())


def _case(seed=31, N=300, frac=0.7):
    wl = W.small_random(n_mesh=(4, 3, 4), L=(8.5, 7.5, 9.0), N=N, seed=seed, species_frac=frac)
    G = W.qround(np.random.default_rng(seed + 1).standard_normal((wl.n, 3)))
    return wl, G


@pytest.mark.parametrize("frac", [None, 0.7])
def test_adjoint_vs_oracle(A, oracle, frac):
    wl, G = _case(frac=frac)
    gam = 0.1
    rx, re, rs, rL = oracle.adjoint(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, gam)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-6)):
        gx, ge, gs, L = gpu_adjoint(A, wl, G, gam, prec)
        ex = rel_max(gx, rx)
        ee = np.abs(ge - re).max() / np.abs(re).max()
        es = np.abs(gs - rs).max() / np.abs(rs).max()
        _note(f"adjoint {prec} species={len(wl.eps)}: dx {ex:.2e} deps {ee:.2e} dsig {es:.2e}")
        assert ex < tol and ee < tol and es < tol
        assert abs(L - rL) < (1e-12 if prec == "fp64" else 1e-5) * abs(rL)


@pytest.mark.parametrize("nsp", [3, 5])
def test_adjoint_many_species(A, oracle, nsp):
    """Mixtures of three and five species (the adjoint's general path, whose parameter sums are kept per
    species pair): dL/dx, dL/deps, dL/dsigma and L against the oracle in both precisions."""
    wl, G = _case(frac=None)
    wl.species = np.random.default_rng(40 + nsp).integers(0, nsp, size=wl.n).astype(np.int32)
    wl.eps, wl.sigma = np.linspace(1.0, 0.5, nsp), np.linspace(1.0, 0.85, nsp)
    gam = 0.1
    rx, re, rs, rL = oracle.adjoint(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, gam)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-6)):
        gx, ge, gs, L = gpu_adjoint(A, wl, G, gam, prec)
        ex = rel_max(gx, rx)
        ee = np.abs(ge - re).max() / np.abs(re).max()
        es = np.abs(gs - rs).max() / np.abs(rs).max()
        _note(f"adjoint {prec} species={nsp}: dx {ex:.2e} deps {ee:.2e} dsig {es:.2e}")
        assert ex < tol and ee < tol and es < tol
        assert abs(L - rL) < (1e-12 if prec == "fp64" else 1e-5) * abs(rL)


def test_adjoint_vs_finite_differences(A, oracle):
    """FP64 central differences (h = 1e-6) of the oracle's L for the four parameters and for
    coordinates whose perturbation leaves the pair set unchanged."""
    wl, G = _case(seed=41, N=200)
    gam = 0.1
    h = 1e-6
    for prec, tol in (("fp64", 1e-6), ("fp32", 1e-6)):
        gx, ge, gs, _ = gpu_adjoint(A, wl, G, gam, prec)
        for which, grad in (("eps", ge), ("sigma", gs)):
            for p in range(len(wl.eps)):
                e1, s1, e2, s2 = wl.eps.copy(), wl.sigma.copy(), wl.eps.copy(), wl.sigma.copy()
                (e1 if which == "eps" else s1)[p] += h
                (e2 if which == "eps" else s2)[p] -= h
                fd = (oracle.loss(wl.x, wl.species, e1, s1, wl.rcut, wl.mesh.periodic, G, gam)
                      - oracle.loss(wl.x, wl.species, e2, s2, wl.rcut, wl.mesh.periodic, G, gam)) / (2 * h)
                _note(f"fd {prec} {which}[{p}] fd={fd:.10e} adj={grad[p]:.10e}")
                assert abs(fd - grad[p]) <= tol * abs(fd)
        P0 = len(oracle.pairs(wl.x, wl.rcut, wl.mesh.periodic))
        rng = np.random.default_rng(43)
        rms = np.sqrt((gx ** 2).mean())
        checked = 0
        for _ in range(40):
            a, k = int(rng.integers(wl.n)), int(rng.integers(3))
            xp, xm = wl.x.copy(), wl.x.copy()
            xp[a, k] += h
            xm[a, k] -= h
            if len(oracle.pairs(xp, wl.rcut, wl.mesh.periodic)) != P0 or \
               len(oracle.pairs(xm, wl.rcut, wl.mesh.periodic)) != P0:
                continue
            fd = (oracle.loss(xp, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, gam)
                  - oracle.loss(xm, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, gam)) / (2 * h)
            assert abs(fd - gx[a, k]) <= max(tol, 1e-6) * max(rms, abs(fd)), (prec, a, k, fd, gx[a, k])
            checked += 1
        assert checked >= 20


@pytest.mark.parametrize("nsp", [2, 3])
def test_autograd_gradcheck(A, nsp):
    import torch
    wl = W.small_random(n_mesh=(3, 3, 3), L=(7.0, 7.0, 7.0), N=40, seed=51, species_frac=0.6, min_sep=0.9)
    if nsp == 3:
        wl.species = np.random.default_rng(52).integers(0, 3, size=wl.n).astype(np.int32)
        wl.eps, wl.sigma = np.array([1.0, 0.5, 0.75]), np.array([1.0, 0.88, 0.94])
    d = A.DIL(wl.mesh, wl.rcut)
    x = torch.tensor(wl.x, dtype=torch.float64, device="cuda", requires_grad=True)
    eps = torch.tensor(wl.eps, dtype=torch.float64, requires_grad=True)
    sig = torch.tensor(wl.sigma, dtype=torch.float64, requires_grad=True)
    sp = torch.tensor(wl.species, dtype=torch.int32, device="cuda")

    def f(x_, e_, s_):
        F, U = A.AicaLJ.apply(x_, e_, s_, d, sp, "fp64")
        return F, U

    assert torch.autograd.gradcheck(f, (x, eps, sig), eps=1e-6, atol=1e-5, rtol=1e-4, nondet_tol=0.0)


def test_full_size_identities(A):
    """219,488-molecule binary mixture: translation invariance (sum dL/dx = 0) and eps-homogeneity
    (sum_s eps_s dL/deps_s = L, since L is linear in every eps_ab and eps_ab is homogeneous of degree
    one in (eps_a, eps_b))."""
    wl = W.config4()
    G = wl.extra["G"]
    d = A.DIL(wl.mesh, wl.rcut)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-6)):
        gx, ge, gs, L = gpu_adjoint(A, wl, G, wl.extra["gamma"], prec, dil=d)
        _note(f"config4 adjoint {prec}: sum dL/dx {np.abs(gx.sum(0)).max():.3e}, "
              f"eps-homogeneity {abs((wl.eps * ge).sum() - L) / abs(L):.3e}")
        assert np.abs(gx.sum(0)).max() < tol * np.abs(gx).sum(0).max()
        assert abs((wl.eps * ge).sum() - L) < tol * abs(L)


def test_one_species_with_scaled_parameters(A, oracle):
    # one species with eps and sigma far from 1 (the one-species kernels apply 24 eps once per pass and
    # take sigma^2 from the table): forces, U, W, pair count and the adjoint against the oracle
    import dataclasses

    import torch
    base = W.small_random(n_mesh=(4, 3, 4), L=(8.5, 7.5, 9.0), N=200, seed=37, min_sep=1.4)
    wl = dataclasses.replace(base, eps=np.array([0.7]), sigma=np.array([1.3]))
    G = W.qround(np.random.default_rng(38).standard_normal((wl.n, 3)))
    gam = 0.2
    Fr, Ur, Wr, nr = oracle.forces(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic)
    rx, re, rs, rL = oracle.adjoint(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, gam)
    d = A.DIL(wl.mesh, wl.rcut)
    for prec, dt, tol, tolA in (("fp64", torch.float64, 1e-12, 1e-12), ("fp32", torch.float32, 1e-5, 1e-6)):
        x = torch.tensor(wl.x, dtype=dt, device="cuda")
        A.aica_bin(d, x)
        F, uw, npairs = A.aica_forces(d, x, None, wl.eps, wl.sigma, precision=prec)
        gx, ge, gs = A.aica_forces_adjoint(d, x, torch.tensor(G, dtype=dt, device="cuda"), gam, None, wl.eps,
                                           wl.sigma, precision=prec)
        torch.cuda.synchronize()
        F = F.double().cpu().numpy()
        eF = np.sqrt(((F - Fr) ** 2).sum(1)).max() / np.sqrt((Fr ** 2).sum(1).mean())
        ex = rel_max(gx.double().cpu().numpy(), rx)
        ee = abs(ge.cpu().numpy()[0] - re[0]) / abs(re[0])
        es = abs(gs.cpu().numpy()[0] - rs[0]) / abs(rs[0])
        _note(f"eps 0.7 sigma 1.3 {prec}: e_F {eF:.2e} dU {abs(uw[0].item() - Ur) / abs(Ur):.2e} "
              f"dx {ex:.2e} deps {ee:.2e} dsig {es:.2e}")
        assert int(npairs.cpu()[0]) == nr
        assert eF < tol and ex < tolA and ee < tolA and es < tolA
        assert abs(uw[0].item() - Ur) <= tol * abs(Ur) and abs(uw[1].item() - Wr) <= tol * abs(Wr)


def test_binary_full_size_against_stored_oracle(A):
    """The 219,488-molecule binary mixture at full size against the stored FP64 oracle results (L, the four
    parameter gradients, their central differences at h = 1e-6, dL/dx on 1,024 fixed rows): both
    precisions, element by element."""
    import os

    import torch
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    import make_binary_adjoint as M
    g = M.read()
    wl = W.config4()
    assert wl.n == int(g["n"])
    d = A.DIL(wl.mesh, wl.rcut)
    for prec, tol, tolL in (("fp64", 1e-12, 1e-12), ("fp32", 1e-6, 1e-5)):
        gx, ge, gs, L = gpu_adjoint(A, wl, wl.extra["G"], wl.extra["gamma"], prec, dil=d)
        ex = np.abs(gx[g["rows"]] - g["dLdx"]).max() / g["rms_dLdx_all"]
        ee = np.abs(ge - g["grad_eps"]) / np.abs(g["grad_eps"])
        es = np.abs(gs - g["grad_sigma"]) / np.abs(g["grad_sigma"])
        fe = np.abs(ge - g["fd_eps"]) / np.abs(g["fd_eps"])
        fs = np.abs(gs - g["fd_sigma"]) / np.abs(g["fd_sigma"])
        _note(f"binary {prec}: dL/dx rows {ex:.2e}, deps {ee.max():.2e}, dsigma {es.max():.2e}, "
              f"vs FD {max(fe.max(), fs.max()):.2e}, L {abs(L - g['L']) / abs(g['L']):.2e}")
        assert ex < tol and ee.max() < tol and es.max() < tol, prec
        assert fe.max() < 1e-6 and fs.max() < 1e-6, prec
        assert abs(L - g["L"]) < tolL * abs(g["L"]), prec
