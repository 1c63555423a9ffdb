"""CPU tests of the library's host side: exported symbols, the interaction lists
(bit-exact against the oracle's brute force), and error handling."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_cs_0702131_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def A():
    import paper_cs_0702131_amd as pkg
    pkg.lib()
    return pkg


def test_library_exports_every_declared_symbol(A):
    header = open(os.path.join(ROOT, "include", "aica.h")).read()
    declared = set(re.findall(r"\b(aica_[a-z_]+)\s*\(", header))
    declared -= {"aica_mesh", "aica_params", "aica_info"}
    assert {"aica_build_dil", "aica_bin", "aica_forces", "aica_forces_adjoint"} <= declared
    L = C.CDLL(A._lib.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(L, name), name


def _dil_case(mesh, rcut, guard, A, oracle):
    """Both cell-pair predicates bit-exact against the brute force; the vertex list is a subset."""
    out = {}
    for pred in ("closest", "vertex"):
        d = A.DIL(mesh, rcut, guard, predicate=pred)
        got = A.aica_dil_export(d)
        ref = oracle.dil(mesh, rcut, guard, pred)
        assert np.array_equal(got, ref), (pred, len(got), len(ref))
        d.close()
        out[pred] = got
    closest = {tuple(r) for r in out["closest"]}
    assert all(tuple(r) in closest for r in out["vertex"])
    return out["closest"]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_dil_matches_bruteforce_jittered_periodic(A, oracle, seed):
    wl = W.small_random(n_mesh=(4, 4, 4), L=(8.0, 8.0, 8.0), N=10, seed=seed, mesh_jitter=0.25)
    _dil_case(wl.mesh, 2.5, 2.5e-6, A, oracle)


def test_dil_matches_bruteforce_walls_and_graded(A, oracle):
    xs = W.graded_nodes(9.0, 0.8, 2.0)
    ys = W.uniform_nodes(7.0, 5)
    zs = W.uniform_nodes(8.0, 4)
    m = W.hex_mesh(xs, ys, zs, periodic_axes=(0, 2), shuffle_seed=3)
    m = W.jitter_interior(m, xs, ys, zs, 0.2, np.random.default_rng(4))
    _dil_case(m, 2.5, 2.5e-6, A, oracle)


def test_dil_matches_bruteforce_tets(A, oracle):
    nodes = W.uniform_nodes(7.0, 3)
    m = W.tet_mesh(nodes, nodes, nodes, periodic_axes=(0, 1, 2))
    _dil_case(m, 2.2, 0.0, A, oracle)


def test_dil_matches_bruteforce_deleted_cells(A, oracle):
    nodes = W.uniform_nodes(10.0, 5)
    m = W.hex_mesh(nodes, nodes, W.uniform_nodes(6.0, 3), periodic_axes=(2,))
    c = np.arange(m.n_cells)
    kill = np.isin(c, [6, 7, 8, 11, 12, 13])
    m2 = W.delete_cells(m, kill)
    assert oracle.min_tet_volume(m2) > 0
    _dil_case(m2, 2.5, 2.5e-6, A, oracle)


@pytest.mark.parametrize("ratio,nc", [(1.0, 27), (1.25, 81), (1.914, 125), (2.5, 275)])
def test_dil_counts_uniform_cubes(A, ratio, nc):
    # on axis-aligned unit cubes the closest points of two cells are vertices, so both predicates
    # give the same N_c
    nodes = np.arange(7.0)
    m = W.hex_mesh(nodes, nodes, nodes, periodic_axes=(0, 1, 2), shuffle_seed=5)
    for pred in ("closest", "vertex"):
        d = A.DIL(m, ratio, 0.0, predicate=pred)
        assert d.info()["n_dil"] == m.n_cells * (nc - 1) // 2


def test_vertex_predicate_misses_on_distorted_mesh(A, oracle):
    # strongly jittered hexes: some cell pairs are within range only between face or edge interiors;
    # the vertex predicate drops exactly those (their vertex pairs are all out of range)
    wl = W.small_random(n_mesh=(5, 5, 5), L=(9.0, 9.0, 9.0), N=10, seed=4, mesh_jitter=0.3)
    m = wl.mesh
    dc = {tuple(r) for r in A.aica_dil_export(A.DIL(m, 2.5, 0.0, predicate="closest"))}
    dv = {tuple(r) for r in A.aica_dil_export(A.DIL(m, 2.5, 0.0, predicate="vertex"))}
    missed = dc - dv
    assert dv <= dc and len(missed) > 0
    cv = {}
    for c in range(m.n_cells):
        f = np.nonzero((m.owner == c) | (m.neighbour == c))[0]
        cv[c] = np.unique(np.concatenate([m.face_pts[m.face_off[k]:m.face_off[k + 1]] for k in f]))
    lat = np.asarray(m.periodic).reshape(-1, 3)
    for c, d, n0, n1, n2 in sorted(missed)[:50]:
        T = np.array([n0, n1, n2])[:len(lat)] @ lat if len(lat) else np.zeros(3)
        vd = np.sqrt(((m.points[cv[c]][:, None, :] - m.points[cv[d]][None, :, :] - T) ** 2).sum(-1)).min()
        assert vd >= 2.5
        assert oracle.cell_distance(m, c, d, T) < 2.5


def test_dil_k5(A):
    m = W.hex_mesh(np.arange(6.0), [0.0, 1.0], [0.0, 1.0])
    D = A.aica_dil_export(A.DIL(m, 10.0, 0.0))
    assert [tuple(r[:2]) for r in D] == [(i, j) for i in range(5) for j in range(i + 1, 5)]


def test_errors_mesh_and_rcut(A):
    nodes = W.uniform_nodes(6.0, 3)
    m = W.hex_mesh(nodes, nodes, nodes, periodic_axes=(0, 1, 2))
    with pytest.raises(A.AicaError) as e:
        A.DIL(m, 3.0, 0.0)           # rcut = L/2
    assert e.value.code == A.AICA_E_RCUT
    with pytest.raises(A.AicaError) as e:
        A.DIL(m, -1.0, 0.0)
    assert e.value.code == A.AICA_E_INVAL
    # inverted cell: move an interior vertex far across the cell
    nodes4 = W.uniform_nodes(6.0, 3)
    bad = W.hex_mesh(nodes4, nodes4, nodes4)
    pts = bad.points.copy()
    k = 1 + 4 * (1 + 4 * 1)           # interior vertex (1,1,1)
    pts[k] += np.array([3.5, 3.5, 3.5])
    bad.points = pts
    with pytest.raises(A.AicaError) as e:
        A.DIL(bad, 1.0, 0.0)
    assert e.value.code == A.AICA_E_MESH
    # face index out of range
    broken = W.hex_mesh(nodes4, nodes4, nodes4)
    fp = broken.face_pts.copy()
    fp[0] = 10 ** 6
    broken.face_pts = fp
    with pytest.raises(A.AicaError) as e:
        A.DIL(broken, 1.0, 0.0)
    assert e.value.code == A.AICA_E_MESH
    # non-orthogonal periodic vectors
    skew = W.hex_mesh(nodes4, nodes4, nodes4, periodic_axes=(0, 1))
    skew.periodic = np.array([[6.0, 0.0, 0.0], [1.0, 6.0, 0.0]])
    with pytest.raises(A.AicaError) as e:
        A.DIL(skew, 1.0, 0.0)
    assert e.value.code == A.AICA_E_INVAL


# ---------------------------------------------------------------- referring transforms with a rotation


@pytest.mark.parametrize("seed,jitter", [(7, 0.2), (8, 0.0)])
def test_dil_matches_bruteforce_wedge(A, oracle, seed, jitter):
    # sector of an annulus: the sides are coupled by the rotation about z, z by a translation
    m = W.wedge_mesh(10.0, 16.0, 12, 6.0, 4, 3, 3, jitter, np.random.default_rng(seed))
    d = _dil_case(m, 2.5, 2.5e-6, A, oracle)
    rot_pairs = d[d[:, 2] != 0]
    assert len(rot_pairs) > 0 and set(np.unique(rot_pairs[:, 2])) == {-1, 1}


def test_dil_wedge_far_images_rejected(A, oracle):
    # near the axis the sector two rotations away is in range: the first powers would not suffice
    narrow = W.wedge_mesh(1.5, 6.0, 8, 6.0, 3, 2, 3, 0.0, np.random.default_rng(1))
    assert oracle.far_images(narrow, 2.5, 2.5e-6) > 0
    with pytest.raises(A.AicaError) as e:
        A.DIL(narrow, 2.5)
    assert e.value.code == A.AICA_E_RCUT
    ok = W.wedge_mesh(10.0, 16.0, 12, 6.0, 4, 3, 3, 0.0, np.random.default_rng(1))
    assert oracle.far_images(ok, 2.5, 2.5e-6) == 0
    A.DIL(ok, 2.5).close()


def test_errors_referring_transforms(A):
    m = W.wedge_mesh(10.0, 16.0, 12, 6.0, 4, 3, 3, 0.0, np.random.default_rng(1))
    good = m.rotations.copy()
    cases = [W.rot_z(1.0),                       # infinite order
             W.rot_z(np.pi / 6) * 1.01,          # not orthonormal
             np.diag([1.0, -1.0, 1.0]),          # a reflection
             W.rot_z(np.pi)]                     # its own inverse
    for r in cases:
        m.rotations = np.stack([r, np.eye(3)])
        with pytest.raises(A.AicaError) as e:
            A.DIL(m, 2.5)
        assert e.value.code == A.AICA_E_INVAL
    # a rotation about z and a translation along x do not commute
    m.rotations = good
    m.periodic = np.array([[0.0, 0.0, 0.0], [6.0, 0.0, 0.0]])
    with pytest.raises(A.AicaError) as e:
        A.DIL(m, 2.5)
    assert e.value.code == A.AICA_E_INVAL


class _FakeTensor:
    """A stand-in with the attributes the binding's checks read (no GPU here)."""

    def __init__(self, shape, is_cuda=True, device="cuda:0"):
        self.shape = tuple(shape)
        self.is_cuda = is_cuda
        self.device = device

    def dim(self):
        return len(self.shape)


def test_adjoint_rejects_bad_grad_forces():
    import paper_cs_0702131_amd as pkg
    pos = _FakeTensor((10, 3))
    pkg._check_grad_forces(_FakeTensor((10, 3)), pos)          # accepted
    for bad in (_FakeTensor((10, 3), is_cuda=False, device="cpu"),  # host memory
                _FakeTensor((10, 3), device="cuda:1"),               # another device
                _FakeTensor((9, 3)),                                  # too few rows
                _FakeTensor((10, 2)),                                 # wrong width
                _FakeTensor((30,)),                                   # flat
                np.zeros((10, 3))):                                   # not a tensor
        with pytest.raises(ValueError):
            pkg._check_grad_forces(bad, pos)


def test_params_reject_mismatched_species_tables():
    """eps and sigma are read for every species: tables of different lengths (or not 1-D) are refused before
    the library sees them."""
    import paper_cs_0702131_amd as pkg
    p, keep = pkg._params(2.5, (1.0, 0.5), (1.0, 0.88), "fp32", True)
    assert p.n_species == 2
    for eps, sig in (((1.0, 0.5), (1.0,)), ((1.0,), (1.0, 0.88)), (np.ones((2, 2)), np.ones((2, 2)))):
        with pytest.raises(ValueError):
            pkg._params(2.5, eps, sig, "fp64", True)
