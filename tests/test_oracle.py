"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
closed forms, lattice sums, crystallographic shell counts, the paper's worked
DIL example, geometric special cases, invariants and brute force."""
import math
import os

import numpy as np
import pytest

from paper_cs_0702131_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden_closed_forms():
    vals = {}
    for line in open(os.path.join(GOLD, "lj_closed_forms.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


# ---------------------------------------------------------------- LJ closed forms (P1)


def test_lj_closed_forms(oracle):
    g = _golden_closed_forms()
    rmin = 2.0 ** (1.0 / 6.0)
    u, gg = oracle.lj(1.0)
    assert abs(u - g["U_at_sigma"]) < 1e-14
    assert abs(gg * 1.0 - g["F_at_sigma"]) < 1e-12          # |F| = g r at r = sigma
    u, gg = oracle.lj(rmin * rmin)
    assert abs(u - g["U_at_rmin"]) < 1e-14
    assert abs(gg * rmin - g["F_at_rmin"]) < 1e-13
    u, gg = oracle.lj(6.25)
    assert abs(u - g["U_at_rcut"]) < 5e-9
    assert abs(gg * 2.5 - g["F_at_rcut"]) < 5e-9
    # U''(r_min) from a central difference of U(r)
    h = 2e-5
    upp = (oracle.lj((rmin + h) ** 2)[0] - 2 * oracle.lj(rmin ** 2)[0] + oracle.lj((rmin - h) ** 2)[0]) / h ** 2
    assert abs(upp - g["U_second_derivative_at_rmin"]) < 5e-6


def test_lj_mixing_and_scaling(oracle):
    # Lorentz-Berthelot on a two-molecule system: eps_ab = sqrt(eps_a eps_b), sigma_ab = mean
    x = np.array([[1.0, 1.0, 1.0], [2.1, 1.3, 0.8]])
    d = x[0] - x[1]
    s = d @ d
    eps, sig = np.array([1.0, 0.5]), np.array([1.0, 0.88])
    F, U, Wv, npairs = oracle.forces(x, [0, 1], eps, sig, 2.5, np.zeros((0, 3)))
    e_ab, s_ab = math.sqrt(0.5), 0.94
    # u(r) = 4 eps ((s/r)^12 - (s/r)^6) at the mixed parameters, via the single-species call
    u1, g1 = oracle.lj(s / s_ab ** 2)          # eps = sigma = 1 at scaled distance
    assert npairs == 1
    assert abs(U - e_ab * u1) < 1e-13
    assert np.allclose(F[0], e_ab * g1 / s_ab ** 2 * d, rtol=1e-13, atol=0)
    assert np.allclose(F[0] + F[1], 0.0, atol=1e-14)
    assert abs(Wv - e_ab * g1 / s_ab ** 2 * s) < 1e-13


def test_two_molecules_across_periodic_face(oracle):
    L = 10.0
    lat = np.eye(3) * L
    x = np.array([[0.3, 5.0, 5.0], [9.6, 5.0, 5.0]])      # 0.7 apart through x = 0
    F, U, Wv, npairs = oracle.forces(x, [0, 0], [1.0], [1.0], 2.5, lat)
    u, g = oracle.lj(0.7 ** 2)
    assert npairs == 1
    assert abs(U - u) < 1e-13 * abs(u)
    assert np.allclose(F[0], [g * 0.7, 0, 0], rtol=1e-12)
    assert np.allclose(F[1], [-g * 0.7, 0, 0], rtol=1e-12)
    # three molecules: a chain through the corner image
    x3 = np.array([[0.2, 0.2, 0.2], [9.9, 9.9, 9.9], [5.0, 5.0, 5.0]])
    F3, U3, _, n3 = oracle.forces(x3, [0, 0, 0], [1.0], [1.0], 2.5, lat)
    d = np.array([0.3, 0.3, 0.3])
    u, g = oracle.lj(d @ d)
    assert n3 == 1 and abs(U3 - u) < 1e-13 * abs(u)
    assert np.allclose(F3[0], g * d, rtol=1e-12) and np.allclose(F3[2], 0)


# ---------------------------------------------------------------- FCC lattice sums (P3)

FCC_SHELLS = [(1, 12), (2, 6), (3, 24), (4, 12), (5, 24), (6, 8), (7, 48), (8, 6)]   # (k, count) at a*sqrt(k/2)


def _fcc_closed_form(a, rc):
    U = Wv = 0.0
    nb = 0
    for k, cnt in FCC_SHELLS:
        r = a * math.sqrt(k / 2.0)
        if r < rc:
            sr6 = r ** -6
            U += 0.5 * cnt * 4.0 * (sr6 * sr6 - sr6)
            Wv += 0.5 * cnt * 24.0 * (2.0 * sr6 * sr6 - sr6)     # g(s) s = 24 (2 r^-12 - r^-6)
            nb += cnt
    return U, Wv, nb


def test_fcc_lattice_sum_matches_shells(oracle):
    L = 10.08
    a = L / 6
    x = W.fcc_sites((6, 6, 6), a)
    F, U, Wv, npairs = oracle.forces(x, np.zeros(len(x), np.int32), [1.0], [1.0], 2.5, np.eye(3) * L)
    Uc, Wc, nb = _fcc_closed_form(a, 2.5)
    N = len(x)
    assert N == 864 and nb == 54 and npairs == 54 * N // 2 == 23328
    assert abs(U / N - Uc) < 1e-12 * abs(Uc)
    assert abs(Wv / N - Wc) < 1e-12 * abs(Wc)
    # the values quoted for this lattice (closed-form lattice sum at a = 1.68)
    assert abs(U / N - (-6.7680388585)) < 1e-9
    assert abs(Wv / N - (-22.1794622011)) < 1e-9
    assert np.abs(F).max() < 1e-12   # inversion symmetry


# ---------------------------------------------------------------- invariants


def test_newton_and_min_image(oracle):
    wl = W.small_random(N=150, seed=11, species_frac=0.7)
    lat = wl.mesh.periodic
    F, U, Wv, npairs = oracle.forces(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, lat)
    scale = np.abs(F).sum()
    assert np.abs(F.sum(axis=0)).max() < 1e-14 * scale
    # minimum image written independently (rc < L/2)
    L = np.diag(lat)
    x = wl.x
    d = x[:, None, :] - x[None, :, :]
    d -= np.round(d / L) * L
    s = (d ** 2).sum(-1)
    np.fill_diagonal(s, np.inf)
    sp = wl.species
    e = np.sqrt(wl.eps[sp][:, None] * wl.eps[sp][None, :])
    sg = 0.5 * (wl.sigma[sp][:, None] + wl.sigma[sp][None, :])
    inr = s < wl.rcut ** 2
    sr6 = np.where(inr, (sg * sg / s) ** 3, 0.0)
    g = np.where(inr, 24 * e * (2 * sr6 * sr6 - sr6) / s, 0.0)
    u = np.where(inr, 4 * e * (sr6 * sr6 - sr6), 0.0)
    Fm = (g[:, :, None] * d).sum(1)
    assert np.allclose(F, Fm, rtol=0, atol=1e-12 * np.abs(Fm).max())
    assert abs(U - 0.5 * u.sum()) < 1e-12 * abs(U)
    assert npairs == inr.sum() // 2


def test_pairs_bruteforce(oracle):
    wl = W.small_random(N=60, seed=3)
    P = oracle.pairs(wl.x, wl.rcut, wl.mesh.periodic)
    L = np.diag(wl.mesh.periodic)
    ref = []
    for a in range(len(wl.x)):
        for b in range(a + 1, len(wl.x)):
            for n in np.ndindex(3, 3, 3):
                n = np.array(n) - 1
                d = wl.x[a] - wl.x[b] - n * L
                if d @ d < wl.rcut ** 2:
                    ref.append((a, b, *n))
    ref = np.array(sorted(ref), dtype=np.int64)
    assert np.array_equal(P, ref)
    _, _, _, npairs = oracle.forces(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic)
    assert npairs == len(P)


# ---------------------------------------------------------------- geometry pins


def test_cell_distance_special_cases(oracle):
    nodes = np.arange(4.0)
    m = W.hex_mesh(nodes, nodes, nodes)           # 3x3x3 unit cubes, cell i + 3 j + 9 k
    c = lambda i, j, k: i + 3 * (j + 3 * k)
    assert oracle.cell_distance(m, c(0, 0, 0), c(1, 0, 0)) == 0.0
    assert abs(oracle.cell_distance(m, c(0, 0, 0), c(2, 0, 0)) - 1.0) < 1e-15
    assert abs(oracle.cell_distance(m, c(0, 0, 0), c(2, 2, 0)) - math.sqrt(2)) < 1e-15
    assert abs(oracle.cell_distance(m, c(0, 0, 0), c(2, 2, 2)) - math.sqrt(3)) < 1e-15
    assert abs(oracle.cell_distance(m, c(0, 0, 0), c(2, 1, 0)) - 1.0) < 1e-15
    # shifted copy: cell (0,0,0) vs cell (2,0,0) moved by +10 x -> gap 11
    assert abs(oracle.cell_distance(m, c(0, 0, 0), c(2, 0, 0), (10.0, 0, 0)) - 11.0) < 1e-13
    # edge-to-edge skew configuration: cube at (0,0,0) vs cube (2,0,2) shifted (0, 0.5, 0)
    assert abs(oracle.cell_distance(m, c(0, 0, 0), c(2, 0, 2), (0, 0.5, 0)) - math.sqrt(2)) < 1e-14


def _two_tets(A, B):
    """A mesh of two separate tetrahedral cells with vertices A[4] and B[4] (every face a boundary face,
    loops oriented out of their cell)."""
    pts = np.concatenate([np.asarray(A, float), np.asarray(B, float)])
    loops, owner = [], []
    for cell in range(2):
        tv = [4 * cell + k for k in range(4)]
        for (a, b, c, d) in ((0, 1, 2, 3), (0, 1, 3, 2), (0, 2, 3, 1), (1, 2, 3, 0)):
            tri = [tv[a], tv[b], tv[c]]
            nrm = np.cross(pts[tri[1]] - pts[tri[0]], pts[tri[2]] - pts[tri[0]])
            if np.dot(nrm, pts[tv[d]] - pts[tri[0]]) > 0:
                tri = tri[::-1]
            loops.append(tri)
            owner.append(cell)
    F = len(owner)
    return W.Mesh(points=pts, face_off=np.arange(F + 1, dtype=np.int64) * 3,
                  face_pts=np.array(loops, dtype=np.int32).ravel(), owner=np.array(owner, np.int32),
                  neighbour=np.full(F, -1, np.int32), n_cells=2)


def _rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    return q if np.linalg.det(q) > 0 else -q


def test_cell_distance_skew_edges(oracle):
    """Two tetrahedra whose closest points are interior points of two skew edges (the edge (0,0,0)-(2,0,0)
    of one, the edge (1,-1,h)-(1,1,h) of the other): the distance is h, and no vertex, no vertex-face foot
    point and no edge end comes closer (the nearest of those is sqrt(1 + h^2) away).  The configuration is
    turned by generic rotations, so no coordinate axis helps.  Sec. 2.2: closest approach of two cells."""
    for h in (0.25, 0.5, 1.7):
        A = [(0, 0, 0), (2, 0, 0), (1, 1, -2), (1, -1, -2)]
        B = [(1, -1, h), (1, 1, h), (0, 0, h + 2), (2, 0, h + 2)]
        for seed in (0, 1, 2):
            R = _rotation(seed)
            m = _two_tets(np.asarray(A, float) @ R.T, np.asarray(B, float) @ R.T)
            assert abs(oracle.cell_distance(m, 0, 1) - h) < 1e-12 * (1 + h), (h, seed)
            # the same through the transform argument (cell 1 moved back by R^T, then forward again)
            m2 = _two_tets(np.asarray(A, float) @ R.T, np.asarray(B, float))
            assert abs(oracle.cell_distance(m2, 0, 1, rot=R) - h) < 1e-12 * (1 + h), (h, seed)


def test_cell_distance_vertex_over_face_interior(oracle):
    """A vertex of one tetrahedron straight above an interior point of a face of the other, along the
    face's normal at height h (the foot (1.7, 0.9) lies inside one of the face's fan triangles, away from
    the fan's spokes): the distance is h; the nearest edge of that face is farther than 0.45.  Generic
    rotations again.  Sec. 2.2: closest approach of two cells."""
    for h in (0.2, 0.6, 1.3):
        A = [(0, 0, 0), (4, 0, 0), (0, 4, 0), (0.5, 0.5, -3)]
        p = np.array([1.7, 0.9, h])
        B = [p, p + (1, 0.2, 3), p + (-0.3, 1, 3), p + (-0.8, -0.9, 3)]
        for seed in (3, 4, 5):
            R = _rotation(seed)
            m = _two_tets(np.asarray(A, float) @ R.T, np.asarray(B, float) @ R.T)
            assert abs(oracle.cell_distance(m, 0, 1) - h) < 1e-12 * (1 + h), (h, seed)


def test_cell_distance_random_tets_against_convex_program(oracle):
    """Separated random tetrahedra: the closest distance of two convex cells is the minimum of
    |sum l_i a_i - sum m_j b_j| over the two simplices of weights, solved here as a small convex program
    (scipy SLSQP), independent of the oracle's triangle-pair routines."""
    from scipy.optimize import minimize
    rng = np.random.default_rng(77)
    for trial in range(40):
        A = rng.uniform(-1, 1, (4, 3))
        B = rng.uniform(-1, 1, (4, 3)) + rng.uniform(-1, 1, 3) * 0 + np.array([rng.uniform(2.2, 3.5), 0, 0])
        R = _rotation(100 + trial)
        A, B = A @ R.T, B @ R.T
        if abs(np.dot(np.cross(A[1] - A[0], A[2] - A[0]), A[3] - A[0])) < 0.05:
            continue
        if abs(np.dot(np.cross(B[1] - B[0], B[2] - B[0]), B[3] - B[0])) < 0.05:
            continue
        m = _two_tets(A, B)

        def f(w):
            d = w[:4] @ A - w[4:] @ B
            return d @ d

        def jac(w):
            d = w[:4] @ A - w[4:] @ B
            return np.concatenate([2 * A @ d, -2 * B @ d])

        cons = [{"type": "eq", "fun": lambda w: w[:4].sum() - 1, "jac": lambda w: np.r_[np.ones(4), np.zeros(4)]},
                {"type": "eq", "fun": lambda w: w[4:].sum() - 1, "jac": lambda w: np.r_[np.zeros(4), np.ones(4)]}]
        best = np.inf
        for start in range(4):
            w0 = np.full(8, 0.25)
            w0[start] += 0.5
            w0[:4] /= w0[:4].sum()
            r = minimize(f, w0, jac=jac, bounds=[(0, 1)] * 8, constraints=cons, method="SLSQP",
                         options={"ftol": 1e-15, "maxiter": 500})
            best = min(best, r.fun)
        ref = np.sqrt(max(best, 0.0))
        got = oracle.cell_distance(m, 0, 1)
        assert abs(got - ref) < 1e-6, (trial, got, ref)


def test_point_location_uniform(oracle):
    nodes = np.linspace(0, 6.0, 4)
    m = W.hex_mesh(nodes, nodes, nodes, shuffle_seed=4)
    base = W.hex_mesh(nodes, nodes, nodes)
    rng = np.random.default_rng(5)
    x = rng.uniform(0.01, 5.99, size=(300, 3))
    ijk = np.floor(x / 2.0).astype(int)
    struct = ijk[:, 0] + 3 * (ijk[:, 1] + 3 * ijk[:, 2])
    # shuffled index of structured cell s: owner of the same face in both meshes
    new_of_old = np.zeros(27, int)
    new_of_old[base.owner] = m.owner
    got = oracle.locate(m, x)
    assert np.array_equal(got, new_of_old[struct])
    # outside the mesh -> -1
    assert oracle.locate(m, np.array([[7.0, 1.0, 1.0]]))[0] == -1
    # on a shared face: lowest index of the two cells wins
    p = np.array([[2.0, 1.0, 1.0]])
    a, b = new_of_old[0], new_of_old[1]
    assert oracle.locate(m, p)[0] == min(a, b)


def test_jittered_mesh_is_valid_and_located(oracle):
    wl = W.small_random(N=200, seed=9)
    assert oracle.min_tet_volume(wl.mesh) > 0
    cells = oracle.locate(wl.mesh, wl.x)
    assert (cells >= 0).all()


# ---------------------------------------------------------------- DIL pins (P5, P6)


def _nc_closed_form(ratio):
    r2 = ratio * ratio
    cnt = 0
    for a in range(-5, 6):
        for b in range(-5, 6):
            for c in range(-5, 6):
                s = sum(max(abs(v) - 1, 0) ** 2 for v in (a, b, c))
                if s < r2:
                    cnt += 1
    return cnt


@pytest.mark.parametrize("ratio,nc", [(1.0, 27), (1.25, 81), (1.5625, 117), (1.914, 125), (2.0, 125), (2.5, 275)])
def test_dil_counts_on_uniform_cubes(oracle, ratio, nc):
    assert _nc_closed_form(ratio) == nc
    nodes = np.arange(7.0)          # 6^3 unit cubes, periodic
    m = W.hex_mesh(nodes, nodes, nodes, periodic_axes=(0, 1, 2), shuffle_seed=2)
    D = oracle.dil(m, ratio, 0.0)
    assert len(D) == m.n_cells * (nc - 1) // 2
    # the paper's vertex-to-vertex predicate gives the same lists on axis-aligned cubes (Sec. 2.4)
    assert np.array_equal(oracle.dil(m, ratio, 0.0, "vertex"), D)
    # no cell on its own list with a zero image; (c,c,n) only with n > 0
    same = D[D[:, 0] == D[:, 1]]
    assert not np.any((same[:, 2:] == 0).all(axis=1))
    assert np.all(D[:, 0] <= D[:, 1])


def test_dil_k5_worked_example(oracle):
    table = {}
    for line in open(os.path.join(GOLD, "dil_k5_table.txt")):
        if line.startswith("#") or not line.strip():
            continue
        i, js = line.split(":")
        table[int(i)] = [int(v) for v in js.split()]
    m = W.hex_mesh(np.arange(6.0), [0.0, 1.0], [0.0, 1.0])    # 5 cubes in a row, all within rc = 10
    D = oracle.dil(m, 10.0, 0.0)
    got = {i: [] for i in range(5)}
    for c, d, *_ in D:
        got[int(c)].append(int(d))
    assert got == table


def test_dil_contains_every_interacting_pair(oracle):
    # every molecule pair in range lies in the same cell or in a DIL cell pair (coverage)
    wl = W.small_random(n_mesh=(4, 4, 4), L=(8.0, 8.0, 8.0), N=180, seed=21)
    D = oracle.dil(wl.mesh, wl.rcut, 1e-6 * wl.rcut)
    cells = oracle.locate(wl.mesh, wl.x)
    P = oracle.pairs(wl.x, wl.rcut, wl.mesh.periodic)
    keys = set(map(tuple, D.tolist()))
    for a, b, n0, n1, n2 in P:
        ca, cb = int(cells[a]), int(cells[b])
        n = (int(n0), int(n1), int(n2))
        if ca == cb and n == (0, 0, 0):
            continue
        # pair d = x_a - x_b - n.L ; cell pair (ca, cb, n) or its mirror (cb, ca, -n)
        k1 = (ca, cb, *n)
        k2 = (cb, ca, *(-v for v in n))
        assert k1 in keys or k2 in keys


# ---------------------------------------------------------------- adjoint pins (P10)


def _adj_case():
    wl = W.small_random(N=120, seed=31, species_frac=0.7)
    G = W.qround(np.random.default_rng(32).standard_normal((wl.n, 3)))
    return wl, G


def test_adjoint_parameter_fd(oracle):
    wl, G = _adj_case()
    gam = 0.1
    gx, ge, gs, L = oracle.adjoint(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, gam)
    L0 = oracle.loss(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, gam)
    assert abs(L - L0) < 1e-12 * abs(L0)
    h = 1e-6
    for which, grad in (("eps", ge), ("sigma", gs)):
        for p in range(len(wl.eps)):
            e1, s1 = wl.eps.copy(), wl.sigma.copy()
            e2, s2 = wl.eps.copy(), wl.sigma.copy()
            if which == "eps":
                e1[p] += h; e2[p] -= h
            else:
                s1[p] += h; s2[p] -= h
            fd = (oracle.loss(wl.x, wl.species, e1, s1, wl.rcut, wl.mesh.periodic, G, gam)
                  - oracle.loss(wl.x, wl.species, e2, s2, wl.rcut, wl.mesh.periodic, G, gam)) / (2 * h)
            assert abs(fd - grad[p]) < 1e-6 * max(1.0, abs(grad[p])), (which, p, fd, grad[p])
    # eps-homogeneity: sum_t eps_t dL/deps_t = L
    assert abs((wl.eps * ge).sum() - L) < 1e-10 * abs(L)


def test_adjoint_parameter_fd_three_species(oracle):
    """Three species under Lorentz-Berthelot: the oracle's parameter gradients (summed per species pair and
    taken back through the mixing rule) against central differences of L from its force routine, and
    eps-homogeneity (L is linear in every eps_ab, so sum_t eps_t dL/deps_t = L)."""
    wl, G = _adj_case()
    wl.species = np.random.default_rng(33).integers(0, 3, size=wl.n).astype(np.int32)
    wl.eps, wl.sigma = np.array([1.0, 0.5, 0.8]), np.array([1.0, 0.88, 0.95])
    gam = 0.1
    gx, ge, gs, L = oracle.adjoint(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, gam)
    h = 1e-6
    for which, grad in (("eps", ge), ("sigma", gs)):
        for p in range(3):
            e1, s1 = wl.eps.copy(), wl.sigma.copy()
            e2, s2 = wl.eps.copy(), wl.sigma.copy()
            if which == "eps":
                e1[p] += h; e2[p] -= h
            else:
                s1[p] += h; s2[p] -= h
            fd = (oracle.loss(wl.x, wl.species, e1, s1, wl.rcut, wl.mesh.periodic, G, gam)
                  - oracle.loss(wl.x, wl.species, e2, s2, wl.rcut, wl.mesh.periodic, G, gam)) / (2 * h)
            assert abs(fd - grad[p]) < 1e-6 * max(1.0, abs(grad[p])), (which, p, fd, grad[p])
    assert abs((wl.eps * ge).sum() - L) < 1e-10 * abs(L)


def test_adjoint_position_fd_and_invariants(oracle):
    wl, G = _adj_case()
    gam = 0.1
    gx, ge, gs, L = oracle.adjoint(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, gam)
    assert np.abs(gx.sum(axis=0)).max() < 1e-12 * np.abs(gx).sum()
    h = 1e-6
    P0 = oracle.pairs(wl.x, wl.rcut, wl.mesh.periodic)
    rng = np.random.default_rng(33)
    checked = 0
    for _ in range(24):
        a, k = int(rng.integers(wl.n)), int(rng.integers(3))
        xp, xm = wl.x.copy(), wl.x.copy()
        xp[a, k] += h
        xm[a, k] -= h
        if len(oracle.pairs(xp, wl.rcut, wl.mesh.periodic)) != len(P0) or \
           len(oracle.pairs(xm, wl.rcut, wl.mesh.periodic)) != len(P0):
            continue
        fd = (oracle.loss(xp, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, gam)
              - oracle.loss(xm, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, gam)) / (2 * h)
        assert abs(fd - gx[a, k]) < 1e-6 * max(1.0, np.sqrt((gx ** 2).mean())), (a, k, fd, gx[a, k])
        checked += 1
    assert checked >= 16


def test_adjoint_rows(oracle):
    # the sampled-row adjoint used at sizes the full adjoint cannot reach: with G = 0 it is gamma grad U
    # = -gamma F on those rows (forces pinned on their own), and for any G it is the full adjoint's rows
    wl, G = _adj_case()
    rows = np.array([0, 7, 7, 119, 53])
    F = oracle.forces_rows(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, rows)[0]
    g0 = oracle.adjoint_rows(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic,
                             np.zeros_like(G), 0.5, rows)
    assert np.allclose(g0, -0.5 * F, rtol=0, atol=1e-13 * np.abs(F).max())
    gx = oracle.adjoint(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, 0.1)[0]
    gr = oracle.adjoint_rows(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, 0.1, rows)
    assert np.array_equal(gr, gx[rows])
    assert oracle.adjoint_rows(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, 0.1,
                               np.zeros(0, np.int64)).shape == (0, 3)


def test_adjoint_hessian_symmetry(oracle):
    wl, G = _adj_case()
    V = W.qround(np.random.default_rng(34).standard_normal((wl.n, 3)))
    # with gamma = 0 the adjoint is -H G (H the Hessian of U), so <V, adj(G)> = <G, adj(V)>
    ag = oracle.adjoint(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, G, 0.0)[0]
    av = oracle.adjoint(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, V, 0.0)[0]
    lhs, rhs = float((V * ag).sum()), float((G * av).sum())
    assert abs(lhs - rhs) < 1e-11 * max(abs(lhs), 1.0)
    # gamma-only loss is U: adjoint = gamma grad U = -gamma F
    F = oracle.forces(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic)[0]
    a0 = oracle.adjoint(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, wl.mesh.periodic, np.zeros_like(G), 0.5)[0]
    assert np.allclose(a0, -0.5 * F, rtol=0, atol=1e-13 * np.abs(F).max())


# ---------------------------------------------------------------- NVE (P11)


def _verlet_energy_span(oracle, x0, lat, dt, steps):
    x = x0.copy()
    v = np.zeros_like(x)
    sp = np.zeros(len(x), np.int32)
    F, U, _, npairs0 = oracle.forces(x, sp, [1.0], [1.0], 2.5, lat)
    uc = oracle.lj(6.25)[0]
    E0 = U - npairs0 * uc
    span = 0.0
    for _ in range(steps):
        v += 0.5 * dt * F
        x += dt * v
        F, U, _, npairs = oracle.forces(x, sp, [1.0], [1.0], 2.5, lat)
        assert npairs == npairs0   # crossing-free system: the pair set never changes
        v += 0.5 * dt * F
        E = 0.5 * (v ** 2).sum() + U - npairs * uc
        span = max(span, abs(E - E0))
    return span


def test_nve_energy_error_scales_dt2(oracle):
    wl = W.fcc_cube(10.08, 4, 6, jitter=0.02, seed=41)
    lat = wl.mesh.periodic
    T = 0.2
    s1 = _verlet_energy_span(oracle, wl.x, lat, 0.004, int(T / 0.004))
    s2 = _verlet_energy_span(oracle, wl.x, lat, 0.002, int(T / 0.002))
    ratio = s1 / s2
    assert 3.2 < ratio < 4.8, ratio


# ---------------------------------------------------------------- rotational referral (Sec. 2.2.2)
#
# Pins of the referring transform with a rotation: the paper's formula for R against the plane
# rotation about z built from cos / sin, and the sector oracle (images under the sector rotation and
# the z translation) against the whole annulus assembled from rotated copies and evaluated with z
# translations only, so that no rotation of the oracle enters the reference side.


def _boundary_face_normals(mesh, pred):
    """Unit outward normals and centres of the boundary faces whose centre satisfies pred."""
    out = []
    for f in range(mesh.n_faces):
        if mesh.neighbour[f] >= 0:
            continue
        loop = mesh.face_pts[mesh.face_off[f]:mesh.face_off[f + 1]]
        P = mesh.points[loop]
        c = P.mean(0)
        if not pred(c):
            continue
        n = np.cross(P[1] - P[0], P[2] - P[0])
        out.append((n / np.linalg.norm(n), c))
    return out


def test_referring_transform_formula(oracle):
    # antiparallel normals (a plain periodic boundary): R = I, y = C_b - C_a
    R, y = oracle.referring_transform([1, 0, 0], [-1, 0, 0], [5.0, 1, 2], [0.0, 1, 2])
    assert np.allclose(R, np.eye(3), atol=1e-15) and np.allclose(y, [-5, 0, 0], atol=1e-15)
    rng = np.random.default_rng(3)
    for _ in range(20):
        na, nb = rng.standard_normal(3), rng.standard_normal(3)
        na, nb = na / np.linalg.norm(na), nb / np.linalg.norm(nb)
        R, y = oracle.referring_transform(na, nb, rng.standard_normal(3), rng.standard_normal(3))
        assert np.allclose(R @ -na, nb, atol=1e-13)                    # -n_a onto n_b
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-13)             # orthogonal
        assert abs(np.linalg.det(R) - 1.0) < 1e-13                      # proper rotation
        ax = np.cross(na, nb)                                           # the axis stays put
        assert np.allclose(R @ ax, ax, atol=1e-13)
    # the wedge's coupled sides: outward normals of the faces on phi = 0 and on phi = theta
    m = W.wedge_mesh(10.0, 22.0, 12, 8.0, 3, 2, 2, 0.0, np.random.default_rng(0), shuffle=False)
    th = m.wedge["theta"]
    side0 = _boundary_face_normals(m, lambda c: abs(c[1]) < 1e-9)
    side1 = _boundary_face_normals(m, lambda c: abs(c[1] - math.tan(th) * c[0]) < 1e-9 and c[1] > 1e-9)
    assert len(side0) == len(side1) == 3 * 2
    Rz = W.rot_z(th)
    for (na, ca) in side0:
        # the coupled face: the one whose centre is the rotated centre
        nb, cb = min(side1, key=lambda t: np.linalg.norm(t[1] - Rz @ ca))
        R, y = oracle.referring_transform(na, nb, ca, cb)
        assert np.allclose(R, Rz, atol=1e-13)
        assert np.allclose(y, 0.0, atol=1e-12)
        assert np.allclose(y + R @ ca, cb, atol=1e-12)   # the face centre goes to the coupled centre
    # re-referring: two sector rotations compose to the rotation by 2 theta; with a z shift as well
    R2, y2 = oracle.compose_transforms((Rz, np.zeros(3)), (Rz, np.array([0.0, 0.0, 8.0])))
    assert np.allclose(R2, W.rot_z(2 * th), atol=1e-14) and np.allclose(y2, [0, 0, 8.0])
    p = np.array([12.0, 1.0, 3.0])
    assert np.allclose(y2 + R2 @ p, Rz @ (Rz @ p) + [0, 0, 8.0], atol=1e-13)


@pytest.fixture(scope="module")
def wedge_small():
    return W.wedge()


def test_wedge_forces_equal_whole_annulus(oracle, wedge_small):
    w = wedge_small
    K = w.mesh.wedge["n_sectors"]
    F, U, Wv, npairs = oracle.forces(w.x, w.species, w.eps, w.sigma, w.rcut, w.lattice, rot=w.rotations)
    full, xf, _ = W.annulus_from_wedge(w.mesh, w.x)
    Ff, Uf, Wf, nf = oracle.forces(xf, np.zeros(len(xf), np.int32), w.eps, w.sigma, w.rcut, full.periodic)
    n = w.n
    assert npairs > 10 * n // 2 and nf == K * npairs
    assert abs(Uf - K * U) <= 1e-11 * abs(Uf)
    assert abs(Wf - K * Wv) <= 1e-11 * abs(Wf)
    scale = np.sqrt(np.mean(F ** 2))
    assert np.max(np.abs(Ff[:n] - F)) <= 1e-11 * scale
    # every copy carries the rotated forces
    for s in (1, 5):
        Rs = W.rot_z(s * w.mesh.wedge["theta"])
        assert np.max(np.abs(Ff[s * n:(s + 1) * n] - F @ Rs.T)) <= 1e-11 * scale
    # the sector sees molecules across both coupled sides (otherwise the check above is vacuous)
    pr = oracle.pairs(w.x, w.rcut, w.lattice, rot=w.rotations)
    assert (pr[:, 2] == 1).sum() > 20 and (pr[:, 2] == -1).sum() > 20


def test_wedge_torque_and_axial_force_vanish(oracle, wedge_small):
    # rotation about z and translation along z leave (x cross F)_z and F_z of every pair balanced
    w = wedge_small
    F, U, Wv, npairs = oracle.forces(w.x, w.species, w.eps, w.sigma, w.rcut, w.lattice, rot=w.rotations)
    scale = np.abs(F).sum()
    tz = (w.x[:, 0] * F[:, 1] - w.x[:, 1] * F[:, 0]).sum()
    assert abs(tz) <= 1e-12 * scale * 22.0
    assert abs(F[:, 2].sum()) <= 1e-12 * scale
    # while the in-plane net force need not vanish (the system is not translation invariant in x, y)
    assert abs(F[:, 0].sum()) > 1e-6 * scale


def test_wedge_adjoint_equals_whole_annulus(oracle, wedge_small):
    w = wedge_small
    K = w.mesh.wedge["n_sectors"]
    G = np.random.default_rng(5).standard_normal((w.n, 3))
    gx, ge, gs, L = oracle.adjoint(w.x, w.species, w.eps, w.sigma, w.rcut, w.lattice, G, 0.3, rot=w.rotations)
    full, xf, Gf = W.annulus_from_wedge(w.mesh, w.x, G)
    gxf, gef, gsf, Lf = oracle.adjoint(xf, np.zeros(len(xf), np.int32), w.eps, w.sigma, w.rcut, full.periodic,
                                       Gf, 0.3)
    assert abs(Lf - K * L) <= 1e-11 * abs(Lf)
    assert abs(gef[0] - K * ge[0]) <= 1e-11 * abs(gef[0])
    assert abs(gsf[0] - K * gs[0]) <= 1e-11 * abs(gsf[0])
    assert np.max(np.abs(gxf[:w.n] - gx)) <= 1e-11 * np.sqrt(np.mean(gx ** 2))
    # L itself: sum G.F + gamma U from the forces
    F, U, _, _ = oracle.forces(w.x, w.species, w.eps, w.sigma, w.rcut, w.lattice, rot=w.rotations)
    assert abs(L - (np.sum(G * F) + 0.3 * U)) <= 1e-12 * (abs(L) + abs(U))


def test_wedge_adjoint_rows(oracle, wedge_small):
    w = wedge_small
    G = np.random.default_rng(6).standard_normal((w.n, 3))
    gx = oracle.adjoint(w.x, w.species, w.eps, w.sigma, w.rcut, w.lattice, G, 0.3, rot=w.rotations)[0]
    rows = np.arange(0, w.n, 37)
    gr = oracle.adjoint_rows(w.x, w.species, w.eps, w.sigma, w.rcut, w.lattice, G, 0.3, rows, rot=w.rotations)
    assert np.array_equal(gr, gx[rows])


def test_wedge_pairs_map_to_annulus_pairs(oracle, wedge_small):
    w = wedge_small
    K, n = w.mesh.wedge["n_sectors"], w.n
    pr = oracle.pairs(w.x, w.rcut, w.lattice, rot=w.rotations)
    full, xf, _ = W.annulus_from_wedge(w.mesh, w.x)
    pf = oracle.pairs(xf, w.rcut, full.periodic)
    assert len(pf) == K * len(pr)
    # pair (s_a N + a, s_b N + b, z) is the sector pair (a, b) through rotation power s_b - s_a (mod K)
    sa, a = np.divmod(pf[:, 0], n)
    sb, b = np.divmod(pf[:, 1], n)
    rp = np.mod(sb - sa + K // 2, K) - K // 2
    assert np.all(np.abs(rp) <= 1)
    mapped = oracle.canonical_pairs(a, b, np.stack([rp, pf[:, 2], np.zeros_like(rp)], axis=1))
    uniq, cnt = np.unique(mapped, axis=0, return_counts=True)
    assert np.all(cnt == K)
    assert np.array_equal(uniq, pr)


def test_wedge_dil_equals_annulus_dil(oracle):
    m = W.wedge_mesh(10.0, 16.0, 12, 6.0, 4, 3, 3, 0.2, np.random.default_rng(7))
    K = m.wedge["n_sectors"]
    rc, guard = 2.5, 1e-6 * 2.5
    dil = oracle.dil(m, rc, guard)
    full, _, _ = W.annulus_from_wedge(m, np.zeros((0, 3)))
    dfull = oracle.dil(full, rc, guard)
    nc = m.n_cells
    assert len(dfull) == K * len(dil)
    sc, c = np.divmod(dfull[:, 0], nc)
    sd, d = np.divmod(dfull[:, 1], nc)
    rp = np.mod(sd - sc + K // 2, K) - K // 2
    assert np.all(np.abs(rp) <= 1)
    mapped = oracle.canonical_pairs(c, d, np.stack([rp, dfull[:, 2], np.zeros_like(rp)], axis=1))
    uniq, cnt = np.unique(mapped, axis=0, return_counts=True)
    assert np.all(cnt == K)
    assert np.array_equal(uniq, dil)
    assert (dil[:, 2] != 0).sum() > 0
    # the first powers suffice here; near the axis they do not
    assert oracle.far_images(m, rc, guard) == 0
    narrow = W.wedge_mesh(1.5, 6.0, 8, 6.0, 3, 2, 3, 0.0, np.random.default_rng(1))
    assert oracle.far_images(narrow, rc, guard) > 0


def test_invalid_referring_transforms(oracle):
    x = np.array([[11.0, 1.0, 1.0], [12.0, 1.5, 2.0]])
    lat = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 8.0]])
    ok = np.stack([W.rot_z(math.pi / 6), np.eye(3)])
    oracle.forces(x, [0, 0], [1.0], [1.0], 2.5, lat, rot=ok)
    bad = [np.stack([W.rot_z(1.0), np.eye(3)]),                      # infinite order
           np.stack([W.rot_z(math.pi / 6) * 1.01, np.eye(3)]),       # not orthogonal
           np.stack([np.diag([1.0, 1.0, -1.0]), np.eye(3)])]          # a reflection
    for r in bad:
        with pytest.raises(ValueError):
            oracle.forces(x, [0, 0], [1.0], [1.0], 2.5, lat, rot=r)
    # a half turn is its own inverse: its group {I, T} is summed once for the forces, but the cell
    # pairs through powers -1 and 1 would list the same image twice
    half = np.stack([W.rot_z(math.pi), np.eye(3)])
    oracle.forces(x, [0, 0], [1.0], [1.0], 2.5, lat, rot=half)
    m = W.wedge_mesh(10.0, 16.0, 2, 6.0, 2, 2, 2, 0.0, np.random.default_rng(1))
    with pytest.raises(ValueError):
        oracle.dil(m, 2.5, 0.0)
    # rotation about z with a translation along x: the two do not commute
    with pytest.raises(ValueError):
        oracle.forces(x, [0, 0], [1.0], [1.0], 2.5, np.array([[0.0, 0, 0], [30.0, 0, 0]]), rot=ok)


def test_binary_full_size_stored_results():
    """The stored FP64 oracle results of the 219,488-molecule binary mixture (written by
    tests/golden/make_binary_adjoint.py, about 2.3 h of CPU): the analytic parameter gradients agree with
    the central differences of the oracle's loss (h = 1e-6) to 1e-7, they satisfy the eps-homogeneity sum
    rule against the stored L, and the stored rows are the ones the fixed seed draws."""
    import sys
    sys.path.insert(0, GOLD)
    import make_binary_adjoint as M
    g = M.read()
    assert int(g["n"]) == 219488 and len(g["rows"]) == M.NROWS
    assert np.array_equal(g["rows"], M.sample_rows(int(g["n"])))
    for a, f in ((g["grad_eps"], g["fd_eps"]), (g["grad_sigma"], g["fd_sigma"])):
        assert np.all(np.abs(a - f) <= 1e-7 * np.abs(f)), (a, f)
    assert np.isfinite(g["dLdx"]).all() and g["rms_dLdx_all"] > 0
    # L is linear in every eps_ab and eps_ab is homogeneous of degree one in the species' eps: with
    # eps = (1, 0.5), sum_s eps_s dL/deps_s = L
    assert abs(1.0 * g["grad_eps"][0] + 0.5 * g["grad_eps"][1] - g["L"]) < 1e-10 * abs(g["L"])
