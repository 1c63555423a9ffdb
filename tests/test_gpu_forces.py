"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Error measures: e_F = max_a |dF_a| / rms_a |F_ref,a|; energies |dU|/|U|.
Bars: FP64 path 1e-12, FP32 path 1e-5; pair sets and pair counts bit-exact."""
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


def eF(F, Fr):
    rms = np.sqrt((Fr ** 2).sum(1).mean())
    return np.sqrt(((F - Fr) ** 2).sum(1)).max() / rms


def run_gpu(A, wl, precision, species=True, compensated=True, dil=None, pos_dtype=None):
    import torch
    d = dil or A.DIL(wl.mesh, wl.rcut)
    pdt = pos_dtype or (torch.float64 if precision == "fp64" else torch.float32)
    x = torch.tensor(wl.x, dtype=pdt, device="cuda")
    sp = torch.tensor(wl.species, dtype=torch.int32, device="cuda") if species else None
    A.aica_bin(d, x)
    F, uw, npairs = A.aica_forces(d, x, sp, wl.eps, wl.sigma, precision=precision, compensated=compensated)
    torch.cuda.synchronize()
    return d, x, F.double().cpu().numpy(), uw.cpu().numpy(), int(npairs.cpu()[0])


def check_case(A, oracle, wl, precision, tolF, tolU, pairs=True):
    _note(f"case {wl.name} n={wl.n} {precision}")
    Fr, Ur, Wr, nr = oracle.forces(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic)
    d, x, F, uw, npairs = run_gpu(A, wl, precision)
    assert npairs == nr
    e = eF(F, Fr)
    assert e < tolF, e
    assert abs(uw[0] - Ur) <= tolU * abs(Ur)
    assert abs(uw[1] - Wr) <= tolU * abs(Wr)
    if pairs:
        P = A.aica_pairs_export(d, x, precision=precision)
        Pr = oracle.pairs(wl.x, wl.rcut, wl.mesh.periodic)
        assert np.array_equal(P, Pr)
    return e


def test_fcc864_fp64(A, oracle):
    check_case(A, oracle, W.config1(), "fp64", 1e-12, 1e-12)


def test_fcc864_fp32(A, oracle):
    check_case(A, oracle, W.config1(), "fp32", 1e-5, 1e-6)


def test_perfect_fcc_lattice_sum(A, oracle):
    wl = W.config1(jitter=0.0)
    d, x, F, uw, npairs = run_gpu(A, wl, "fp64")
    Fr, Ur, Wr, nr = oracle.forces(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic)
    assert npairs == nr == 23328
    # positions are rounded to multiples of 2^-15, so the lattice is perfect only to ~1e-5 and the
    # net forces (~1e-3) are sums of pair forces of order 1..30 that nearly cancel; the FP64 bar is
    # therefore stated against the pair-force scale F(sigma) = 24 eps / sigma
    assert np.abs(F - Fr).max() < 1e-12 * 24.0
    assert np.abs(F).max() < 1e-2
    assert abs(uw[0] - Ur) < 1e-12 * abs(Ur)


@pytest.mark.parametrize("seed,periodic,species", [(1, (0, 1, 2), None), (2, (0, 2), 0.7), (3, (1,), 0.5),
                                                   (4, (), None)])
def test_small_random_both_precisions(A, oracle, seed, periodic, species):
    wl = W.small_random(n_mesh=(4, 3, 5), L=(8.5, 7.0, 9.0), N=300, periodic_axes=periodic, seed=seed,
                        species_frac=species)
    check_case(A, oracle, wl, "fp64", 1e-12, 1e-12)
    check_case(A, oracle, wl, "fp32", 1e-5, 1e-6)


@pytest.mark.parametrize("nsp", [3, 8])
def test_many_species(A, oracle, nsp):
    """Mixtures of three and eight species (the largest the library takes; parameters looked up per pair
    from the Lorentz-Berthelot table): forces, U, W and the pair set against the oracle in both precisions."""
    wl = W.small_random(n_mesh=(4, 3, 5), L=(8.5, 7.0, 9.0), N=300, seed=70 + nsp)
    wl.species = np.random.default_rng(80 + nsp).integers(0, nsp, size=wl.n).astype(np.int32)
    wl.eps, wl.sigma = np.linspace(1.0, 0.4, nsp), np.linspace(1.0, 0.8, nsp)
    check_case(A, oracle, wl, "fp64", 1e-12, 1e-12)
    check_case(A, oracle, wl, "fp32", 1e-5, 1e-6)


@pytest.mark.parametrize("seed,periodic", [(5, (0, 1, 2)), (6, (1,))])
def test_pair_counts_per_molecule(A, oracle, seed, periodic):
    """aica_pair_counts against the oracle's pair list: every pair counts once for each member, a molecule
    paired with its own image twice; both precisions, caller order."""
    wl = W.small_random(n_mesh=(4, 3, 5), L=(8.5, 7.0, 9.0), N=300, periodic_axes=periodic, seed=seed,
                        species_frac=0.5)
    P = oracle.pairs(wl.x, wl.rcut, wl.mesh.periodic)
    ref = np.bincount(P[:, 0], minlength=wl.n) + np.bincount(P[:, 1], minlength=wl.n)
    for prec in ("fp64", "fp32"):
        d, x, _, _, npairs = run_gpu(A, wl, prec)
        counts = A.aica_pair_counts(d, x, precision=prec).cpu().numpy()
        assert np.array_equal(counts, ref), prec
        assert npairs == len(P)


def test_cutoff_band_pairs(A, oracle):
    # separations within a few FP32 ulps of rc^2 on both sides (and exactly rc): the FP32 path must
    # reproduce the exact pair set, including pairs where a plain FP32 evaluation of s decides wrongly
    wl = W.cutoff_band_pairs()
    n = wl.n // 2
    d = wl.x[n:] - wl.x[:n]
    d -= wl.box_hi[0] * np.round(d / wl.box_hi[0])
    m = np.round(d / W.Q).astype(np.int64)
    exact_in = (m ** 2).sum(1) < int(round(2.5 / W.Q)) ** 2
    d32 = d.astype(np.float32)
    t = np.float32(d32[:, 2].astype(np.float64) ** 2)  # fmaf(dx, dx, fmaf(dy, dy, dz * dz))
    t = np.float32(d32[:, 1].astype(np.float64) ** 2 + t)
    s32 = np.float32(d32[:, 0].astype(np.float64) ** 2 + t)
    assert ((s32 < np.float32(6.25)) != exact_in).sum() > 0
    for prec in ("fp32", "fp64"):
        check_case(A, oracle, wl, prec, 1e-5 if prec == "fp32" else 1e-12, 1e-5 if prec == "fp32" else 1e-12)


def test_dense_coarse_mesh_many_chunks(A, oracle):
    # 2x2x2 cells of 4.2 sigma at density ~0.8: ~60 molecules per cell, so groups of more than 64
    # molecules (several i-passes), j-lists of several segments and ragged tails everywhere
    wl = W.small_random(n_mesh=(2, 2, 2), L=(8.4, 8.4, 8.4), N=470, seed=8, min_sep=0.85, species_frac=0.8)
    check_case(A, oracle, wl, "fp64", 1e-12, 1e-12)
    check_case(A, oracle, wl, "fp32", 1e-5, 1e-6)


@pytest.mark.parametrize("L,n_fcc,frac", [(13.44, 8, None), (18.48, 11, 0.6)])
def test_cells_beyond_a_segment(A, oracle, L, n_fcc, frac):
    """A 2x2x2 periodic mesh of cells holding 256 or 665-666 molecules each (an FCC fluid at density 0.845):
    every cell is larger than a j segment in both precisions (at most 240 expanded j), so neighbour cells
    are split across segments and groups need four to eleven passes.  Forces, U, W, the pair set, the
    per-molecule pair counts and the adjoint against the oracle in both precisions."""
    import torch
    wl = W.fcc_cube(L, 2, n_fcc, jitter=0.05, seed=int(10 * L), name=f"fcc{4 * n_fcc ** 3}_mesh2")
    if frac is not None:
        rng = np.random.default_rng(int(10 * L) + 1)
        wl.species = (rng.random(wl.n) < frac).astype(np.int32)
        wl.eps, wl.sigma = np.array([1.0, 0.7]), np.array([1.0, 0.9])
    d0 = A.DIL(wl.mesh, wl.rcut)
    A.aica_bin(d0, torch.tensor(wl.x, dtype=torch.float64, device="cuda"))
    _, _, count = A.aica_bin_export(d0, wl.n)
    assert count.sum() == wl.n and count.min() >= wl.n // 8 > 240
    check_case(A, oracle, wl, "fp64", 1e-12, 1e-12)
    check_case(A, oracle, wl, "fp32", 1e-5, 1e-6)
    P = oracle.pairs(wl.x, wl.rcut, wl.mesh.periodic)
    ref = np.bincount(P[:, 0], minlength=wl.n) + np.bincount(P[:, 1], minlength=wl.n)
    G = W.qround(np.random.default_rng(int(10 * L) + 2).standard_normal((wl.n, 3)))
    rx, re, rs, _ = oracle.adjoint(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, 0.1)
    for prec, dt, tol in (("fp64", torch.float64, 1e-12), ("fp32", torch.float32, 1e-6)):
        xt = torch.tensor(wl.x, dtype=dt, device="cuda")
        sp = torch.tensor(wl.species, dtype=torch.int32, device="cuda")
        A.aica_bin(d0, xt)
        counts = A.aica_pair_counts(d0, xt, precision=prec).cpu().numpy()
        assert np.array_equal(counts, ref), prec
        gx, ge, gs = A.aica_forces_adjoint(d0, xt, torch.tensor(G, dtype=dt, device="cuda"), 0.1, sp, wl.eps,
                                           wl.sigma, precision=prec)
        gx = gx.double().cpu().numpy()
        ex = np.abs(gx - rx).max() / np.sqrt((rx ** 2).mean())
        ee = np.abs(ge.cpu().numpy() - re).max() / np.abs(re).max()
        es = np.abs(gs.cpu().numpy() - rs).max() / np.abs(rs).max()
        _note(f"  {wl.name} adjoint {prec}: dx {ex:.2e} deps {ee:.2e} dsig {es:.2e}")
        assert ex < tol and ee < tol and es < tol, prec


def test_edge_cases_tiny(A, oracle):
    import torch
    wl = W.small_random(N=2, seed=9, min_sep=0)
    for n in (0, 1, 2):
        sub = W.Workload("tiny", wl.mesh, wl.x[:n].copy(), wl.species[:n].copy(), wl.eps, wl.sigma, wl.rcut,
                         wl.box_lo, wl.box_hi, wl.periodic_axes)
        d, x, F, uw, npairs = run_gpu(A, sub, "fp64")
        Fr, Ur, Wr, nr = oracle.forces(sub.x, sub.species, sub.eps, sub.sigma, sub.rcut, sub.mesh.periodic)
        assert npairs == nr
        assert F.shape == (n, 3)
        if n:
            assert np.allclose(F, Fr, rtol=1e-12, atol=1e-12)
        assert abs(uw[0] - Ur) <= 1e-12 * max(abs(Ur), 1e-300)


def test_mesh_independence(A, oracle):
    """Same molecules on different meshes (uniform, jittered, finer, tetrahedral): identical pair
    sets and FP64 forces (the paper's third verification criterion)."""
    L = float(W.qround(8.0))
    base = W.small_random(n_mesh=(4, 4, 4), L=(L, L, L), N=260, seed=12, mesh_jitter=0.0)
    nodes4, nodes8 = W.uniform_nodes(L, 4), W.uniform_nodes(L, 8)
    meshes = [base.mesh,
              W.jitter_interior(W.hex_mesh(nodes4, nodes4, nodes4, periodic_axes=(0, 1, 2)), nodes4, nodes4, nodes4,
                                0.25, np.random.default_rng(3)),
              W.hex_mesh(nodes8, nodes8, nodes8, periodic_axes=(0, 1, 2), shuffle_seed=9),
              W.tet_mesh(W.uniform_nodes(L, 3), W.uniform_nodes(L, 3), W.uniform_nodes(L, 3), periodic_axes=(0, 1, 2))]
    ref = None
    for m in meshes:
        wl = W.Workload("meshind", m, base.x, base.species, base.eps, base.sigma, 2.5, base.box_lo, base.box_hi,
                        (0, 1, 2))
        d, x, F, uw, npairs = run_gpu(A, wl, "fp64")
        P = A.aica_pairs_export(d, x, precision="fp64")
        if ref is None:
            ref = (F, uw, P)
            Fr = oracle.forces(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, m.periodic)[0]
            assert eF(F, Fr) < 1e-12
        else:
            assert np.array_equal(P, ref[2])
            assert eF(F, ref[0]) < 1e-12
            assert abs(uw[0] - ref[1][0]) < 1e-12 * abs(ref[1][0])


def test_binning_against_oracle(A, oracle):
    import torch
    wl = W.small_random(n_mesh=(4, 4, 4), L=(8.0, 8.0, 8.0), N=400, seed=14)
    d = A.DIL(wl.mesh, 2.5)
    x = torch.tensor(wl.x, device="cuda")
    A.aica_bin(d, x)
    cell_of, order, count = A.aica_bin_export(d, wl.n)
    assert np.array_equal(cell_of, oracle.locate(wl.mesh, wl.x))
    assert np.array_equal(count, np.bincount(cell_of, minlength=wl.mesh.n_cells))
    assert np.array_equal(np.sort(order), np.arange(wl.n))
    # molecules grouped by cell, ascending id inside each cell
    co = cell_of[order]
    starts = np.flatnonzero(np.r_[True, co[1:] != co[:-1]])
    assert len(starts) == len(np.unique(co))
    for s, e in zip(starts, np.r_[starts[1:], wl.n]):
        assert np.all(np.diff(order[s:e]) > 0)


def test_unlocated_and_call_order_errors(A):
    import torch
    wl = W.small_random(N=50, seed=15, periodic_axes=(0, 2))
    d = A.DIL(wl.mesh, 2.5)
    xb = wl.x.copy()
    xb[3, 1] = 100.0                         # outside the walls
    xt = torch.tensor(xb, device="cuda")
    with pytest.raises(A.AicaError) as e:
        A.aica_bin(d, xt)
    assert e.value.code == A.AICA_E_UNLOCATED
    xb[3, 1] = float("nan")
    with pytest.raises(A.AicaError) as e:
        A.aica_bin(d, torch.tensor(xb, device="cuda"))
    assert e.value.code == A.AICA_E_UNLOCATED
    x = torch.tensor(wl.x, device="cuda")
    A.aica_bin(d, x)
    other = x.clone()
    with pytest.raises(A.AicaError) as e:
        A.aica_forces(d, other, None, [1.0], [1.0], precision="fp64")
    assert e.value.code == A.AICA_E_INVAL


def test_deterministic_repeat(A):
    import torch
    wl = W.config1()
    d, x, F1, uw1, n1 = run_gpu(A, wl, "fp32")
    F2, uw2, n2 = A.aica_forces(d, x, None, wl.eps, wl.sigma, precision="fp32")
    assert np.array_equal(F1, F2.double().cpu().numpy())
    assert np.array_equal(uw1, uw2.cpu().numpy())


def test_config2_walls_jittered(A, oracle):
    wl = W.config2()
    e64 = check_case(A, oracle, wl, "fp64", 1e-12, 1e-12)
    e32 = check_case(A, oracle, wl, "fp32", 1e-5, 1e-6)
    _note(f"config2 e_F fp64={e64:.3e} fp32={e32:.3e}")


def test_config4_full_size_sampled_rows(A, oracle):
    """219,488-molecule binary mixture at full size: the FP32 and FP64 forces on 600 sampled
    rows against the oracle (each row summed over all molecules), exact pair counts on those rows,
    and zero net force."""
    wl = W.config4()
    rows = np.random.default_rng(40).choice(wl.n, 600, replace=False)
    Fr, Ur, Wr, cnt = oracle.forces_rows(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, rows)
    rms = np.sqrt((Fr ** 2).sum(1).mean())
    d = A.DIL(wl.mesh, wl.rcut)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        _, x, F, uw, npairs = run_gpu(A, wl, prec, dil=d)
        err = np.sqrt(((F[rows] - Fr) ** 2).sum(1)).max() / rms
        _note(f"config4 {prec} sampled e_F = {err:.3e}, npairs = {npairs}")
        assert err < tol, err
        assert abs(F.sum(0)).max() < (1e-9 if prec == "fp64" else 1e-2) * np.abs(F).sum(0).max()
        counts = A.aica_pair_counts(d, x, precision=prec).cpu().numpy()
        assert np.array_equal(counts[rows], cnt), prec
        assert int(counts.sum()) == 2 * npairs


def test_binning_tracking_after_moves(A, oracle):
    """Second binning with molecules moved (some across cell faces, some onto a shared face):
    the previous-cell fast path must give the same cells as brute-force location."""
    import torch
    wl = W.small_random(n_mesh=(4, 4, 4), L=(8.0, 8.0, 8.0), N=400, seed=16)
    d = A.DIL(wl.mesh, 2.5)
    x0 = torch.tensor(wl.x, device="cuda")
    A.aica_bin(d, x0)
    rng = np.random.default_rng(17)
    x1 = wl.x + W.qround(rng.uniform(-0.6, 0.6, size=wl.x.shape))
    x1 = np.mod(x1, 8.0)
    x1 = W.qround(x1)
    x1 = np.where(x1 >= 8.0, x1 - 8.0, x1)
    x1[:5] = [[2.0, 2.0, 2.0], [4.0, 1.0, 1.0], [0.0, 3.0, 5.0], [6.0, 6.0, 6.0], [1.0, 4.0, 2.0]]  # mesh planes
    t1 = torch.tensor(x1, device="cuda")
    A.aica_bin(d, t1)
    cell_of, order, count = A.aica_bin_export(d, wl.n)
    ref = oracle.locate(wl.mesh, x1)
    assert np.array_equal(cell_of, ref)
    F, uw, npairs = A.aica_forces(d, t1, None, [1.0], [1.0], precision="fp64")
    Fr, Ur, Wr, nr = oracle.forces(x1, np.zeros(wl.n, np.int32), [1.0], [1.0], 2.5, wl.mesh.periodic)
    assert int(npairs.item()) == nr
    assert eF(F.cpu().numpy(), Fr) < 1e-12


@pytest.mark.parametrize("cfg", ["config2", "config4"])
def test_vertex_predicate_missed_pairs(A, oracle, cfg):
    """The paper's vertex-to-vertex cell predicate against the closest-distance lists on the jittered
    meshes: the pairs it finds are a subset; the pairs it misses are counted (printed)."""
    import torch
    wl = getattr(W, cfg)()
    x = torch.tensor(wl.x, dtype=torch.float64, device="cuda")
    keys, cells = {}, {}
    for pred in ("closest", "vertex"):
        d = A.DIL(wl.mesh, wl.rcut, predicate=pred)
        A.aica_bin(d, x)
        P = A.aica_pairs_export(d, x, precision="fp64")
        code = 9 * (P[:, 2] + 1) + 3 * (P[:, 3] + 1) + (P[:, 4] + 1)
        keys[pred] = (P[:, 0] << 40) | (P[:, 1] << 12) | code
        cells[pred] = d.info()["n_dil"]
        d.close()
    assert np.all(np.isin(keys["vertex"], keys["closest"]))
    missed = len(keys["closest"]) - len(keys["vertex"])
    _note(f"{wl.name}: cell pairs closest {cells['closest']} vertex {cells['vertex']}; molecule pairs "
          f"{len(keys['closest'])}, missed by the vertex predicate {missed} ({missed / len(keys['closest']):.2e})")
    if cfg == "config2":
        Pr = oracle.pairs(wl.x, wl.rcut, wl.mesh.periodic)
        assert len(Pr) == len(keys["closest"])


def test_binning_ties_on_faces_edges_vertices(A, oracle):
    """Molecules exactly on shared faces, edges and vertices of an unjittered mesh with shuffled cell
    ids: the lowest containing cell wins, on the first binning (no history), on a repeat (every
    molecule starts from its previous cell) and after moving onto other boundaries."""
    import torch
    L = 8.0
    nodes = W.uniform_nodes(L, 4)
    mesh = W.hex_mesh(nodes, nodes, nodes, periodic_axes=(0, 1, 2), shuffle_seed=21)
    rng = np.random.default_rng(22)
    g = np.arange(4) * 2.0
    pts = []
    for _ in range(300):
        p = rng.uniform(0.1, L - 0.1, size=3)
        k = rng.integers(1, 4)                        # 1, 2 or 3 coordinates on grid planes
        axes = rng.choice(3, size=k, replace=False)
        p[axes] = g[rng.integers(0, 4, size=k)]
        pts.append(p)
    x = W.qround(np.array(pts))
    d = A.DIL(mesh, 2.5)
    for step in range(3):
        if step == 2:
            x = np.roll(x, 1, axis=0)                 # every molecule jumps to another boundary point
        t = torch.tensor(x, device="cuda")
        A.aica_bin(d, t)
        cell_of, order, count = A.aica_bin_export(d, len(x))
        assert np.array_equal(cell_of, oracle.locate(mesh, x)), step


def test_binning_balls_and_routes(A, oracle):
    """Tracking (the paper's membership kept from step to step): the first binning searches and gives each
    molecule that the plane test shows well inside its cell a ball inside that cell; the second finds those
    in their balls and tests the rest against their previous cell's record (which keeps a ball too); the
    third (same positions) needs no geometry at all; small moves then mix the routes, and a molecule that
    crossed a face is mostly located by the record of the cell across it.  Every binning equals brute-force
    location, and the routes add up to n."""
    import torch
    wl = W.small_random(n_mesh=(5, 4, 5), L=(10.0, 8.0, 10.0), N=500, seed=31, mesh_jitter=0.25)
    d = A.DIL(wl.mesh, wl.rcut)
    x = wl.x.copy()
    rng = np.random.default_rng(32)
    routes, cells = [], []
    for step in range(6):
        if step >= 3:  # moves of up to 0.15 per axis, wrapped into the periodic box
            x = W.qround(W.wrap(x + rng.uniform(-0.15, 0.15, size=x.shape), wl.box_lo, wl.box_hi,
                                wl.periodic_axes))
            x = np.minimum(x, wl.box_hi - W.Q)
        t = torch.tensor(x, device="cuda")
        A.aica_bin(d, t)
        cell_of, _, _ = A.aica_bin_export(d, len(x))
        assert np.array_equal(cell_of, oracle.locate(wl.mesh, x)), step
        cells.append(cell_of)
        inf = d.info()
        r = (inf["located_ball"], inf["located_record"], inf["located_search"])
        routes.append(r)
        assert sum(r) == len(x), (step, r)
    _note(f"routes (ball, record, search) per binning: {routes}")
    assert routes[0] == (0, 0, len(x))
    assert routes[1][0] >= 0.5 * len(x) and routes[1][0] + routes[1][1] >= 0.95 * len(x)
    assert routes[2][0] >= 0.95 * len(x)
    assert routes[5][0] > 0 and routes[5][1] + routes[5][2] > 0
    # a molecule that crossed a face is mostly found by the FP32 record of the cell across the face it
    # most likely crossed, without the slow path
    moved = int((cells[5] != cells[4]).sum())
    _note(f"molecules that changed cells in the last move: {moved}; slow path: {routes[5][2]}")
    assert moved > 20 and routes[5][2] < 0.5 * moved


def test_binning_slow_path_lane_groups(A, oracle):
    """The slow location kernel takes a molecule on 16 lanes (four per wave) when the previous binning sent
    more molecules down the slow path than its grid has waves (8,192), else on a whole wave.  12,000 molecules
    at random on a jittered, shuffled mesh: the first binning searches for every one of them, so the second
    (after moves of up to 0.9 per axis, so that many molecules land in cells that are not across a face)
    runs the 16-lane groups, and the third (small moves) whole waves unless the second sent more than 8,192
    molecules down the slow path.  Every binning equals brute-force location, in both position precisions."""
    import torch
    Ls = [float(W.qround(v)) for v in (36.0, 24.0, 30.0)]
    nodes = [W.uniform_nodes(Ls[a], n) for a, n in enumerate((18, 12, 15))]
    mesh = W.jitter_interior(W.hex_mesh(*nodes, periodic_axes=(0, 1, 2)), *nodes, 0.25,
                             np.random.default_rng(41))
    mesh = W.renumber_cells(mesh, np.random.default_rng(42).permutation(mesh.n_cells))
    hi = np.array(Ls)
    rng = np.random.default_rng(43)
    x0 = W.qround(rng.uniform(0.0, 1.0, size=(12000, 3)) * hi)
    x0 = np.minimum(x0, hi - W.Q)
    for dt in (torch.float64, torch.float32):
        d = A.DIL(mesh, 2.5)
        x = x0.copy()
        slow = []
        for step, amp in enumerate((0.0, 0.9, 0.05)):
            if amp > 0:
                x = W.qround(W.wrap(x + rng.uniform(-amp, amp, size=x.shape), np.zeros(3), hi, (0, 1, 2)))
                x = np.minimum(x, hi - W.Q)
            A.aica_bin(d, torch.tensor(x, dtype=dt, device="cuda"))
            cell_of, _, _ = A.aica_bin_export(d, len(x))
            assert np.array_equal(cell_of, oracle.locate(mesh, x)), (dt, step)
            slow.append(d.info()["located_search"])
        d.close()
        _note(f"slow-path molecules per binning ({dt}): {slow}")
        assert slow[0] == len(x0) > 8192  # so the second binning takes the 16-lane groups
        assert slow[1] > 0  # ... and gives them work


def test_cells_at_the_occupancy_limit(A, oracle):
    """Eight cells of 190 molecules each: in the FP64 forward (segments of 192 expanded j) a neighbour
    cell never fits beside the j carried over from the previous segment, so segment boundaries take the
    path that first evaluates the carried j on their own, and neighbour cells are split across segments;
    groups hold one cell, i.e. three passes of up to 64."""
    import torch
    L, per = 14.0, 190
    sites = []
    for ci in range(2):
        for cj in range(2):
            for ck in range(2):
                a, b, c = np.meshgrid(np.arange(6), np.arange(6), np.arange(7), indexing="ij")
                s = np.stack([ci * 7 + 0.55 + a.ravel() * (7.0 / 6.0), cj * 7 + 0.55 + b.ravel() * (7.0 / 6.0),
                              ck * 7 + 0.5 + c.ravel() * 1.0], axis=1)[:per]
                sites.append(s)
    x = np.vstack(sites)
    x = W.qround(x + np.random.default_rng(61).uniform(-0.1, 0.1, size=x.shape))
    nodes = W.uniform_nodes(L, 2)
    mesh = W.hex_mesh(nodes, nodes, nodes, periodic_axes=(0, 1, 2), shuffle_seed=62)
    n = len(x)
    wl = W.Workload("limit", mesh, x, np.zeros(n, np.int32), np.array([1.0]), np.array([1.0]), 2.5,
                    np.zeros(3), np.full(3, L), (0, 1, 2))
    d, _, _, _, _ = run_gpu(A, wl, "fp64")
    _, _, count = A.aica_bin_export(d, n)
    assert count.max() == per and count.min() == per
    check_case(A, oracle, wl, "fp64", 1e-12, 1e-12)
    # U/N is only -0.07 here (close repulsive and attractive pairs nearly cancel), so the FP32 pair
    # energies' relative error of ~1e-7 shows up amplified in U: the bar is 2e-5 of |U| for this case
    check_case(A, oracle, wl, "fp32", 1e-5, 2e-5)
    G = W.qround(np.random.default_rng(63).standard_normal((n, 3)))
    rx, _, _, _ = oracle.adjoint(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, 0.1)
    for prec, dt, tol in (("fp64", torch.float64, 1e-12), ("fp32", torch.float32, 1e-6)):
        xt = torch.tensor(wl.x, dtype=dt, device="cuda")
        A.aica_bin(d, xt)
        gx, _, _ = A.aica_forces_adjoint(d, xt, torch.tensor(G, dtype=dt, device="cuda"), 0.1, None, wl.eps,
                                         wl.sigma, precision=prec)
        gx = gx.double().cpu().numpy()
        assert np.abs(gx - rx).max() / np.sqrt((rx ** 2).mean()) < tol, prec
