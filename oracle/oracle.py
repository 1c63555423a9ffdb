"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  The oracle shares no code with the HIP library; see oracle.c for the
definitions it implements.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99"]


def build(force=False):
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        subprocess.check_call(["gcc", *CFLAGS, "-o", LIB + ".tmp", SRC, "-lm"])
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        p = C.c_void_p
        i64, i32, f64 = C.c_int64, C.c_int32, C.c_double
        L.oc_forces.argtypes = [i64, p, p, i32, p, p, f64, i32, p, p, p, p, p, p]
        L.oc_forces.restype = C.c_int
        L.oc_forces_rows.argtypes = [i64, p, p, i32, p, p, f64, i32, p, p, i64, p, p, p, p, p]
        L.oc_forces_rows.restype = C.c_int
        L.oc_pairs.argtypes = [i64, p, f64, i32, p, p, i64, p, p, p]
        L.oc_pairs.restype = i64
        L.oc_adjoint.argtypes = [i64, p, p, i32, p, p, f64, i32, p, p, p, f64, p, p, p, p]
        L.oc_adjoint.restype = C.c_int
        L.oc_adjoint_rows.argtypes = [i64, p, p, i32, p, p, f64, i32, p, p, p, f64, i64, p, p]
        L.oc_adjoint_rows.restype = C.c_int
        mesh_args = [i64, p, i64, p, p, p, p, i64]
        L.oc_dil.argtypes = mesh_args + [i32, p, p, f64, f64, i32, i64, p, p, p]
        L.oc_dil.restype = i64
        L.oc_far_images.argtypes = mesh_args + [i32, p, p, f64, f64]
        L.oc_far_images.restype = i64
        L.oc_locate.argtypes = mesh_args + [i64, p, p]
        L.oc_locate.restype = C.c_int
        L.oc_cell_distance.argtypes = mesh_args + [i32, i32, p, p]
        L.oc_cell_distance.restype = f64
        L.oc_min_tet_volume.argtypes = mesh_args
        L.oc_min_tet_volume.restype = f64
        L.oc_lj.argtypes = [f64, f64, f64, p, p]
        L.oc_lj.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _lat(lattice, rot=None):
    """Referring transforms x -> R_k x + y_k: lattice [k,3] holds y_k, rot [k,3,3] the R_k (None: R_k = I).
    Returns (y, R, k) as contiguous arrays, R being None when every R_k is the identity."""
    lat = _c(np.asarray(lattice, dtype=np.float64).reshape(-1, 3), np.float64)
    if len(lat) == 0:
        return np.zeros((1, 3)), None, 0
    if rot is not None:
        rot = _c(np.asarray(rot, dtype=np.float64).reshape(len(lat), 3, 3), np.float64)
    return lat, rot, len(lat)


def _rp(rot):
    return None if rot is None else _ptr(rot)


def lj(s, eps=1.0, sigma=1.0):
    """(u, g) of one pair at squared distance s; force on a from b is g * d."""
    u, g = C.c_double(), C.c_double()
    lib().oc_lj(float(s), float(eps), float(sigma), C.byref(u), C.byref(g))
    return u.value, g.value


def forces(x, species, eps, sigma, rcut, lattice, rot=None):
    """All-pairs, all-images FP64 forces [N,3], U, W, npairs."""
    x = _c(x, np.float64)
    n = len(x)
    sp = _c(species, np.int32)
    eps, sig = _c(eps, np.float64), _c(sigma, np.float64)
    lat, rot, nper = _lat(lattice, rot)
    F = np.zeros((n, 3))
    U, W, npairs = C.c_double(), C.c_double(), C.c_int64()
    rc = lib().oc_forces(n, _ptr(x), _ptr(sp), len(eps), _ptr(eps), _ptr(sig), float(rcut), nper, _ptr(lat),
                         _rp(rot), _ptr(F), C.byref(U), C.byref(W), C.byref(npairs))
    if rc != 0:
        raise ValueError(f"oc_forces failed ({rc})")
    return F, U.value, W.value, npairs.value


def forces_rows(x, species, eps, sigma, rcut, lattice, rows, rot=None):
    """Forces on the given rows (each against all molecules); per-row half U, W and pair counts."""
    x = _c(x, np.float64)
    sp = _c(species, np.int32)
    eps, sig = _c(eps, np.float64), _c(sigma, np.float64)
    lat, rot, nper = _lat(lattice, rot)
    rows = _c(rows, np.int64)
    F = np.zeros((len(rows), 3))
    Ur, Wr, cnt = np.zeros(len(rows)), np.zeros(len(rows)), np.zeros(len(rows), np.int64)
    rc = lib().oc_forces_rows(len(x), _ptr(x), _ptr(sp), len(eps), _ptr(eps), _ptr(sig), float(rcut), nper,
                              _ptr(lat), _rp(rot), len(rows), _ptr(rows), _ptr(F), _ptr(Ur), _ptr(Wr), _ptr(cnt))
    if rc != 0:
        raise ValueError(f"oc_forces_rows failed ({rc})")
    return F, Ur, Wr, cnt


def pairs(x, rcut, lattice, rot=None):
    """Canonical pair set: rows (a, b, n0, n1, n2), a < b (a == b: a molecule and its own image, n
    lexicographically positive), sorted."""
    x = _c(x, np.float64)
    lat, rot, nper = _lat(lattice, rot)
    cnt = lib().oc_pairs(len(x), _ptr(x), float(rcut), nper, _ptr(lat), _rp(rot), 0, None, None, None)
    if cnt < 0:
        raise ValueError("oc_pairs failed")
    a, b = np.zeros(cnt, np.int32), np.zeros(cnt, np.int32)
    nn = np.zeros((cnt, 3), np.int8)
    lib().oc_pairs(len(x), _ptr(x), float(rcut), nper, _ptr(lat), _rp(rot), cnt, _ptr(a), _ptr(b), _ptr(nn))
    return canonical_pairs(a, b, nn)


def canonical_pairs(a, b, nn):
    a, b, nn = np.asarray(a, np.int64), np.asarray(b, np.int64), np.asarray(nn, np.int64).reshape(-1, 3)
    # (a, b, n) and (b, a, -n) are one pair; a == b is kept with n lexicographically positive
    neg = (nn[:, 0] < 0) | ((nn[:, 0] == 0) & ((nn[:, 1] < 0) | ((nn[:, 1] == 0) & (nn[:, 2] < 0))))
    swap = (a > b) | ((a == b) & neg)
    a2, b2 = np.where(swap, b, a), np.where(swap, a, b)
    nn2 = np.where(swap[:, None], -nn, nn)
    key = np.stack([a2, b2, nn2[:, 0], nn2[:, 1], nn2[:, 2]], axis=1)
    order = np.lexsort(key.T[::-1])
    return key[order]


def adjoint(x, species, eps, sigma, rcut, lattice, G, gamma, rot=None):
    """Analytic gradient of L = sum G.F + gamma U: (dL/dx [N,3], dL/deps, dL/dsigma, L)."""
    x = _c(x, np.float64)
    sp = _c(species, np.int32)
    eps, sig = _c(eps, np.float64), _c(sigma, np.float64)
    lat, rot, nper = _lat(lattice, rot)
    G = _c(G, np.float64)
    gx = np.zeros_like(x)
    ge, gs = np.zeros(len(eps)), np.zeros(len(eps))
    L = C.c_double()
    rc = lib().oc_adjoint(len(x), _ptr(x), _ptr(sp), len(eps), _ptr(eps), _ptr(sig), float(rcut), nper, _ptr(lat),
                          _rp(rot), _ptr(G), float(gamma), _ptr(gx), _ptr(ge), _ptr(gs), C.byref(L))
    if rc != 0:
        raise ValueError(f"oc_adjoint failed ({rc})")
    return gx, ge, gs, L.value


def adjoint_rows(x, species, eps, sigma, rcut, lattice, G, gamma, rows, rot=None):
    """dL/dx on the given rows only (each against all molecules and images), [len(rows), 3]."""
    x = _c(x, np.float64)
    sp = _c(species, np.int32)
    eps, sig = _c(eps, np.float64), _c(sigma, np.float64)
    lat, rot, nper = _lat(lattice, rot)
    G = _c(G, np.float64)
    rows = _c(rows, np.int64)
    gx = np.zeros((len(rows), 3))
    rc = lib().oc_adjoint_rows(len(x), _ptr(x), _ptr(sp), len(eps), _ptr(eps), _ptr(sig), float(rcut), nper,
                               _ptr(lat), _rp(rot), _ptr(G), float(gamma), len(rows), _ptr(rows), _ptr(gx))
    if rc != 0:
        raise ValueError(f"oc_adjoint_rows failed ({rc})")
    return gx


def loss(x, species, eps, sigma, rcut, lattice, G, gamma, rot=None):
    F, U, _, _ = forces(x, species, eps, sigma, rcut, lattice, rot)
    return float(np.sum(np.asarray(G) * F) + gamma * U)


def _mesh_args(mesh):
    pts = _c(mesh.points, np.float64)
    fo = _c(mesh.face_off, np.int64)
    fp = _c(mesh.face_pts, np.int32)
    ow = _c(mesh.owner, np.int32)
    ne = _c(mesh.neighbour, np.int32)
    keep = (pts, fo, fp, ow, ne)
    return keep, [len(pts), _ptr(pts), len(ow), _ptr(fo), _ptr(fp), _ptr(ow), _ptr(ne), int(mesh.n_cells)]


def dil(mesh, rcut, guard, predicate="closest"):
    """Brute-force interacting cell pairs as sorted rows (c, d, n0, n1, n2).  predicate "closest": the
    closest distance between the closed cells is below rcut + guard; "vertex": some vertex pair is."""
    keep, args = _mesh_args(mesh)
    lat, rot, nper = _lat(mesh.periodic, getattr(mesh, "rotations", None))
    pr = {"closest": 0, "vertex": 1}[predicate]
    cnt = lib().oc_dil(*args, nper, _ptr(lat), _rp(rot), float(rcut), float(guard), pr, 0, None, None, None)
    if cnt < 0:
        raise ValueError(f"oc_dil failed ({cnt})")
    c, d = np.zeros(cnt, np.int32), np.zeros(cnt, np.int32)
    nn = np.zeros((cnt, 3), np.int8)
    lib().oc_dil(*args, nper, _ptr(lat), _rp(rot), float(rcut), float(guard), pr, cnt, _ptr(c), _ptr(d), _ptr(nn))
    key = np.stack([c, d, nn[:, 0], nn[:, 1], nn[:, 2]], axis=1).astype(np.int64)
    return key[np.lexsort(key.T[::-1])]


def far_images(mesh, rcut, guard):
    """Number of cell pairs in range (closest distance below rcut + guard) through an image with some
    generator power outside {-1, 0, 1}; zero when the first images suffice."""
    keep, args = _mesh_args(mesh)
    lat, rot, nper = _lat(mesh.periodic, getattr(mesh, "rotations", None))
    cnt = lib().oc_far_images(*args, nper, _ptr(lat), _rp(rot), float(rcut), float(guard))
    if cnt < 0:
        raise ValueError(f"oc_far_images failed ({cnt})")
    return int(cnt)


def locate(mesh, x):
    keep, args = _mesh_args(mesh)
    x = _c(x, np.float64)
    cell = np.zeros(len(x), np.int32)
    rc = lib().oc_locate(*args, len(x), _ptr(x), _ptr(cell))
    if rc != 0:
        raise ValueError(f"oc_locate failed ({rc})")
    return cell


def cell_distance(mesh, c, d, shift=(0.0, 0.0, 0.0), rot=None):
    """Closest distance between cell c and cell d mapped by x -> rot x + shift."""
    keep, args = _mesh_args(mesh)
    T = _c(shift, np.float64)
    Rm = None if rot is None else _c(np.asarray(rot).reshape(3, 3), np.float64)
    return lib().oc_cell_distance(*args, int(c), int(d), _ptr(T), _rp(Rm))


def min_tet_volume(mesh):
    keep, args = _mesh_args(mesh)
    return lib().oc_min_tet_volume(*args)


def referring_transform(n_a, n_b, c_a, c_b):
    """The referring transform across a coupled boundary (Sec. 2.2.2): R rotates -n_a onto n_b (outward
    unit normals of the coupled faces), R = -(n_a.n_b) I + (1 + n_a.n_b) k k^T + n_a n_b^T - n_b n_a^T
    with k the unit vector along n_a x n_b; a position P is referred to C_b - R C_a + R P, i.e. the
    generic form y + R P with y = C_b - R C_a.  Antiparallel normals give R = I (a translation).
    Returns (R, y)."""
    n_a, n_b = np.asarray(n_a, np.float64), np.asarray(n_b, np.float64)
    c_a, c_b = np.asarray(c_a, np.float64), np.asarray(c_b, np.float64)
    c = float(n_a @ n_b)
    k = np.cross(n_a, n_b)
    kn = np.linalg.norm(k)
    R = -c * np.eye(3) + np.outer(n_a, n_b) - np.outer(n_b, n_a)
    if kn > 0:
        k = k / kn
        R = R + (1.0 + c) * np.outer(k, k)
    y = c_b - R @ c_a
    return R, y


def compose_transforms(first, second):
    """Referring by `first` = (R, y), then by `second` = (R', y'): P'' = y'* + R'* P with
    y'* = y' + R' y and R'* = R' R (Sec. 2.2.2, re-referring)."""
    (R, y), (R2, y2) = first, second
    return R2 @ R, y2 + R2 @ y
