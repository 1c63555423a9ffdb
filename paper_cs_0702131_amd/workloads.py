"""Seeded synthetic inputs: polyhedral meshes, molecule lattices, species and weights.

This module holds no pair-force arithmetic.  It builds the inputs both the HIP
path and the FP64 oracle consume, so that the two sides see identical data.

Meshes use a face-based polyhedral description (the static unstructured mesh
of Sec. 2.3): points, faces as vertex loops (normal out of the owner cell by
the right-hand rule), owner and neighbour cell per face (neighbour -1 on a
boundary), and the referring transforms of the periodic directions: x -> R x + y
with y in `periodic` and R in `rotations` (None: every R = I, plain lattice
translations).  Cell indices can be shuffled, since a cell's index says nothing
about where it is (Sec. 2.3).

All positions and box lengths are rounded to multiples of Q = 2**-15 so that
differences of coordinates below 512 sigma are exact in FP32 and FP64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

Q = 2.0 ** -15


def qround(x):
    """Round to the nearest multiple of Q (exact in FP32 for |x| < 512)."""
    return np.round(np.asarray(x, dtype=np.float64) / Q) * Q


@dataclass
class Mesh:
    points: np.ndarray          # [P,3] f64
    face_off: np.ndarray        # [F+1] i64
    face_pts: np.ndarray        # [K] i32
    owner: np.ndarray           # [F] i32
    neighbour: np.ndarray       # [F] i32, -1 for boundary faces
    n_cells: int
    periodic: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))  # [k,3] transform shifts y_k
    lo: np.ndarray = None       # domain bounding box (for fixtures)
    hi: np.ndarray = None
    rotations: np.ndarray = None  # [k,3,3] transform rotations R_k, or None for lattice translations

    @property
    def n_faces(self):
        return len(self.owner)


# ----------------------------------------------------------------------------------------------
# structured hex meshes (the generator is structured; nothing downstream relies on it)


def hex_mesh(xs, ys, zs, periodic_axes=(), shuffle_seed=None):
    """Tensor-product hex mesh on node coordinates xs, ys, zs."""
    xs, ys, zs = (np.asarray(a, dtype=np.float64) for a in (xs, ys, zs))
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    PX, PY = nx + 1, ny + 1
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    pts = np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(),
                    Z.transpose(2, 1, 0).ravel()], axis=1)  # index i + PX*(j + PY*k)

    def P(i, j, k):
        return i + PX * (j + PY * k)

    def C(i, j, k):
        return i + nx * (j + ny * k)

    loops, owners, neighs = [], [], []
    # x-faces at node plane i (normal +x: y then z)
    i, j, k = np.meshgrid(np.arange(nx + 1), np.arange(ny), np.arange(nz), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    lp = np.stack([P(i, j, k), P(i, j + 1, k), P(i, j + 1, k + 1), P(i, j, k + 1)], axis=1)
    own = np.where(i > 0, C(np.maximum(i - 1, 0), j, k), C(np.minimum(i, nx - 1), j, k))
    nei = np.where((i > 0) & (i < nx), C(np.minimum(i, nx - 1), j, k), -1)
    lp = np.where((i == 0)[:, None], lp[:, ::-1], lp)
    loops.append(lp); owners.append(own); neighs.append(nei)
    # y-faces at node plane j (normal +y: z then x)
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny + 1), np.arange(nz), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    lp = np.stack([P(i, j, k), P(i, j, k + 1), P(i + 1, j, k + 1), P(i + 1, j, k)], axis=1)
    own = np.where(j > 0, C(i, np.maximum(j - 1, 0), k), C(i, np.minimum(j, ny - 1), k))
    nei = np.where((j > 0) & (j < ny), C(i, np.minimum(j, ny - 1), k), -1)
    lp = np.where((j == 0)[:, None], lp[:, ::-1], lp)
    loops.append(lp); owners.append(own); neighs.append(nei)
    # z-faces at node plane k (normal +z: x then y)
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz + 1), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    lp = np.stack([P(i, j, k), P(i + 1, j, k), P(i + 1, j + 1, k), P(i, j + 1, k)], axis=1)
    own = np.where(k > 0, C(i, j, np.maximum(k - 1, 0)), C(i, j, np.minimum(k, nz - 1)))
    nei = np.where((k > 0) & (k < nz), C(i, j, np.minimum(k, nz - 1)), -1)
    lp = np.where((k == 0)[:, None], lp[:, ::-1], lp)
    loops.append(lp); owners.append(own); neighs.append(nei)

    lp = np.concatenate(loops).astype(np.int32)
    owner = np.concatenate(owners).astype(np.int32)
    neighbour = np.concatenate(neighs).astype(np.int32)
    F = len(owner)
    lengths = np.array([xs[-1] - xs[0], ys[-1] - ys[0], zs[-1] - zs[0]])
    per = np.array([np.eye(3)[a] * lengths[a] for a in periodic_axes]).reshape(-1, 3)
    m = Mesh(points=pts, face_off=np.arange(F + 1, dtype=np.int64) * 4, face_pts=lp.ravel(),
             owner=owner, neighbour=neighbour, n_cells=nx * ny * nz, periodic=per,
             lo=np.array([xs[0], ys[0], zs[0]]), hi=np.array([xs[-1], ys[-1], zs[-1]]))
    m.shape = (nx, ny, nz)
    if shuffle_seed is not None:
        m = renumber_cells(m, np.random.default_rng(shuffle_seed).permutation(m.n_cells))
    return m


def renumber_cells(m: Mesh, new_of_old):
    """Give old cell c the new index new_of_old[c]; faces keep owner as the lower... no: owner stays owner."""
    new_of_old = np.asarray(new_of_old)
    owner = new_of_old[m.owner].astype(np.int32)
    neighbour = np.where(m.neighbour >= 0, new_of_old[np.maximum(m.neighbour, 0)], -1).astype(np.int32)
    out = Mesh(points=m.points, face_off=m.face_off, face_pts=m.face_pts, owner=owner,
               neighbour=neighbour, n_cells=m.n_cells, periodic=m.periodic, lo=m.lo, hi=m.hi,
               rotations=m.rotations)
    return out


def delete_cells(m: Mesh, kill):
    """Remove cells flagged in kill[n_cells]; faces to removed cells become boundary faces."""
    kill = np.asarray(kill, dtype=bool)
    keep_idx = np.cumsum(~kill) - 1
    o_k = ~kill[m.owner]
    n_k = np.where(m.neighbour >= 0, ~kill[np.maximum(m.neighbour, 0)], False)
    offs, pts_list, owners, neighs = [], [], [], []
    fo, fp = m.face_off, m.face_pts
    loops = [fp[fo[f]:fo[f + 1]] for f in range(m.n_faces)] if m.n_faces < 0 else None
    # vectorised for quads and general loops alike
    lens = np.diff(fo)
    keep_face = o_k | n_k
    flip = (~o_k) & n_k
    new_owner = np.where(o_k, m.owner, np.maximum(m.neighbour, 0))
    new_nei = np.where(o_k & n_k, m.neighbour, -1)
    sel = np.nonzero(keep_face)[0]
    new_loops = []
    for f in sel:
        lp = fp[fo[f]:fo[f + 1]]
        new_loops.append(lp[::-1] if flip[f] else lp)
    new_lens = lens[sel]
    face_off = np.concatenate([[0], np.cumsum(new_lens)]).astype(np.int64)
    out = Mesh(points=m.points, face_off=face_off,
               face_pts=np.concatenate(new_loops).astype(np.int32) if new_loops else np.zeros(0, np.int32),
               owner=keep_idx[new_owner[sel]].astype(np.int32),
               neighbour=np.where(new_nei[sel] >= 0, keep_idx[np.maximum(new_nei[sel], 0)], -1).astype(np.int32),
               n_cells=int((~kill).sum()), periodic=m.periodic, lo=m.lo, hi=m.hi, rotations=m.rotations)
    return out


def jitter_interior(m: Mesh, xs, ys, zs, amp, rng):
    """Move every vertex not on the domain boundary by U(-amp*h, amp*h) per axis.

    h is the smaller of the two node spacings adjacent to the vertex along that
    axis.  Boundary vertices stay put, so periodic faces remain translates."""
    xs, ys, zs = (np.asarray(a, dtype=np.float64) for a in (xs, ys, zs))
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    pts = m.points.copy()
    idx = np.arange(len(pts))
    i = idx % (nx + 1)
    j = (idx // (nx + 1)) % (ny + 1)
    k = idx // ((nx + 1) * (ny + 1))
    interior = (i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)

    def local_h(nodes, ii):
        d = np.diff(nodes)
        left = d[np.clip(ii - 1, 0, len(d) - 1)]
        right = d[np.clip(ii, 0, len(d) - 1)]
        return np.minimum(left, right)

    h = np.stack([local_h(xs, i), local_h(ys, j), local_h(zs, k)], axis=1)
    du = rng.uniform(-1.0, 1.0, size=pts.shape) * amp * h
    pts[interior] += du[interior]
    out = Mesh(points=pts, face_off=m.face_off, face_pts=m.face_pts, owner=m.owner,
               neighbour=m.neighbour, n_cells=m.n_cells, periodic=m.periodic, lo=m.lo, hi=m.hi,
               rotations=m.rotations)
    out.shape = getattr(m, "shape", None)
    return out


def tet_mesh(xs, ys, zs, periodic_axes=()):
    """Split every hex of a tensor-product grid into 6 tetrahedra (Kuhn split).

    The split is conforming across neighbouring hexes, so the result is a
    valid tetrahedral mesh of the same box."""
    xs, ys, zs = (np.asarray(a, dtype=np.float64) for a in (xs, ys, zs))
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    PX, PY = nx + 1, ny + 1
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    pts = np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(),
                    Z.transpose(2, 1, 0).ravel()], axis=1)
    tets = []
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                base = np.array([i, j, k])
                for pa in perms:
                    v = [base.copy()]
                    cur = base.copy()
                    for ax in pa:
                        cur = cur.copy(); cur[ax] += 1
                        v.append(cur)
                    tets.append([a[0] + PX * (a[1] + PY * a[2]) for a in v])
    tets = np.array(tets, dtype=np.int64)
    # faces of each tet; orient so the normal points out of the tet
    face_map = {}
    loops, owner, neighbour = [], [], []
    for t, tv in enumerate(tets):
        p = pts[tv]
        vol = np.dot(np.cross(p[1] - p[0], p[2] - p[0]), p[3] - p[0])
        for (a, b, c, d) in ((0, 1, 2, 3), (0, 1, 3, 2), (0, 2, 3, 1), (1, 2, 3, 0)):
            tri = [tv[a], tv[b], tv[c]]
            n = np.cross(pts[tri[1]] - pts[tri[0]], pts[tri[2]] - pts[tri[0]])
            if np.dot(n, pts[tv[d]] - pts[tri[0]]) > 0:
                tri = tri[::-1]
            key = tuple(sorted(tri))
            if key in face_map:
                f = face_map[key]
                neighbour[f] = t
            else:
                face_map[key] = len(owner)
                loops.append(tri); owner.append(t); neighbour.append(-1)
    F = len(owner)
    lengths = np.array([xs[-1] - xs[0], ys[-1] - ys[0], zs[-1] - zs[0]])
    per = np.array([np.eye(3)[a] * lengths[a] for a in periodic_axes]).reshape(-1, 3)
    return Mesh(points=pts, face_off=np.arange(F + 1, dtype=np.int64) * 3,
                face_pts=np.array(loops, dtype=np.int32).ravel(), owner=np.array(owner, np.int32),
                neighbour=np.array(neighbour, np.int32), n_cells=len(tets), periodic=per,
                lo=np.array([xs[0], ys[0], zs[0]]), hi=np.array([xs[-1], ys[-1], zs[-1]]))


def graded_nodes(length, h_edge, h_mid, n=None):
    """Node coordinates on [0, length] graded symmetrically from h_edge at both
    ends to h_mid at the centre (spacing varies linearly with distance from the
    nearer end)."""
    half = length / 2.0
    # spacing h(s) = h_edge + (h_mid - h_edge) * s / half for s in [0, half]
    xs = [0.0]
    while xs[-1] < half:
        s = xs[-1]
        xs.append(s + h_edge + (h_mid - h_edge) * min(s / half, 1.0))
    m = len(xs) - 1
    left = np.array(xs[: m + 1]) * (half / xs[m])
    nodes = np.concatenate([left, length - left[::-1][1:]])
    return nodes


def uniform_nodes(length, n):
    return np.linspace(0.0, length, n + 1)


# ----------------------------------------------------------------------------------------------
# molecules


def fcc_sites(ncell, a, shift=0.25):
    """FCC sites: ncell = (nx,ny,nz) unit cells of edge a = (ax,ay,az), first site at shift*a."""
    nx, ny, nz = ncell
    a = np.broadcast_to(np.asarray(a, dtype=np.float64), (3,))
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]) + shift
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cells = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1).astype(np.float64)
    sites = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    return sites


def wrap(x, lo, hi, periodic_axes):
    x = x.copy()
    for ax in periodic_axes:
        L = hi[ax] - lo[ax]
        x[:, ax] = lo[ax] + np.mod(x[:, ax] - lo[ax], L)
    return x


def soft_relax(x, lo, hi, periodic_axes, steps, rng=None, r0=1.0, step=0.01, clip=0.05):
    """Steepest descent on a harmonic overlap penalty sum (r0 - r)^2 for r < r0.

    This is input preparation (remove close contacts of random positions); it
    is deliberately not the Lennard-Jones model under test."""
    from scipy.spatial import cKDTree
    L = hi - lo
    per = np.zeros(3, bool)
    per[list(periodic_axes)] = True
    x = x.copy()
    for _ in range(steps):
        box = np.where(per, L, 0.0)
        xs = x - lo
        # cKDTree periodic box only for periodic axes: pad non-periodic with a large box
        bs = np.where(per, L, 10.0 * L.max() + 10.0)
        xs_b = np.where(per, np.mod(xs, L), xs + 2.0 * L.max() + 2.0)
        tree = cKDTree(xs_b, boxsize=bs)
        pairs = tree.query_pairs(r0, output_type="ndarray")
        if len(pairs) == 0:
            break
        d = xs_b[pairs[:, 0]] - xs_b[pairs[:, 1]]
        d -= np.where(per, np.round(d / np.where(per, L, 1.0)) * L, 0.0)
        r = np.linalg.norm(d, axis=1)
        r = np.maximum(r, 1e-9)
        f = (2.0 * (r0 - r) / r)[:, None] * d
        F = np.zeros_like(x)
        np.add.at(F, pairs[:, 0], f)
        np.add.at(F, pairs[:, 1], -f)
        x += np.clip(step * F, -clip, clip)
        for ax in range(3):
            if per[ax]:
                x[:, ax] = lo[ax] + np.mod(x[:, ax] - lo[ax], L[ax])
            else:
                # reflect into [lo, hi]
                y = x[:, ax]
                y = np.where(y < lo[ax], 2 * lo[ax] - y, y)
                y = np.where(y > hi[ax], 2 * hi[ax] - y, y)
                x[:, ax] = y
    return x


# ----------------------------------------------------------------------------------------------
# named workloads


@dataclass
class Workload:
    name: str
    mesh: Mesh
    x: np.ndarray                 # [N,3] f64, multiples of Q, inside the mesh
    species: np.ndarray           # [N] i32
    eps: np.ndarray               # [n_species] per-species epsilon
    sigma: np.ndarray             # [n_species] per-species sigma
    rcut: float
    box_lo: np.ndarray
    box_hi: np.ndarray
    periodic_axes: tuple
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return len(self.x)

    @property
    def lattice(self):
        return self.mesh.periodic

    @property
    def rotations(self):
        return self.mesh.rotations


def _rng(k, child):
    return np.random.default_rng([0xA1CA, k, child])


def fcc_cube(L_nominal=10.08, n_mesh=4, n_fcc=6, jitter=0.05, mesh_jitter=0.0, seed=1, shuffle=True,
             name="fcc_cube"):
    """Periodic cube of FCC LJ molecules on a uniform (optionally jittered) hex mesh."""
    L = float(qround(L_nominal))
    nodes = uniform_nodes(L, n_mesh)
    mesh = hex_mesh(nodes, nodes, nodes, periodic_axes=(0, 1, 2))
    if mesh_jitter > 0:
        mesh = jitter_interior(mesh, nodes, nodes, nodes, mesh_jitter, _rng(seed, 0))
    if shuffle:
        mesh = renumber_cells(mesh, _rng(seed, 5).permutation(mesh.n_cells))
    a = L / n_fcc
    x = fcc_sites((n_fcc,) * 3, a)
    if jitter > 0:
        x = x + _rng(seed, 1).uniform(-jitter, jitter, size=x.shape)
    lo, hi = np.zeros(3), np.full(3, L)
    x = wrap(qround(x), lo, hi, (0, 1, 2))
    x = qround(x)
    x = np.where(x >= L, x - L, x)
    return Workload(name, mesh, x, np.zeros(len(x), np.int32), np.array([1.0]), np.array([1.0]), 2.5,
                    lo, hi, (0, 1, 2))


def config1(seed=1, jitter=0.05):
    """Single-species FCC fluid, L=10.08, 4x4x4 uniform hex mesh, N=864, rc=2.5."""
    return fcc_cube(10.08, 4, 6, jitter=jitter, seed=seed, name="fcc864_mesh4")


def config2(seed=2, relax_steps=200, n=None):
    """40x20x20 box periodic in x,z with walls in y; jittered 25x13x13 hex mesh;
    about 13,440 molecules (density 0.84) from uniform random positions relaxed
    by steepest descent on a soft overlap penalty."""
    Lx, Ly, Lz = (float(qround(v)) for v in (40.0, 20.0, 20.0))
    xs, ys, zs = uniform_nodes(Lx, 25), uniform_nodes(Ly, 13), uniform_nodes(Lz, 13)
    mesh = hex_mesh(xs, ys, zs, periodic_axes=(0, 2))
    mesh = jitter_interior(mesh, xs, ys, zs, 0.25, _rng(2, 0))
    mesh = renumber_cells(mesh, _rng(2, 5).permutation(mesh.n_cells))
    N = n if n is not None else int(round(0.84 * 16000))
    lo, hi = np.zeros(3), np.array([Lx, Ly, Lz])
    r = _rng(seed, 1)
    x = lo + r.uniform(0, 1, size=(N, 3)) * (hi - lo)
    x = soft_relax(x, lo, hi, (0, 2), relax_steps)
    x = qround(x)
    x = wrap(x, lo, hi, (0, 2))
    x = qround(x)
    for ax in (0, 2):
        x[:, ax] = np.where(x[:, ax] >= hi[ax], x[:, ax] - (hi[ax] - lo[ax]), x[:, ax])
    x[:, 1] = np.clip(x[:, 1], Q, Ly - Q)
    return Workload("random13440_box40x20x20_jitter", mesh, x, np.zeros(N, np.int32), np.array([1.0]),
                    np.array([1.0]), 2.5, lo, hi, (0, 2))


def binary_species(N, frac_a, rng):
    s = np.ones(N, np.int32)
    s[rng.permutation(N)[: int(round(frac_a * N))]] = 0
    return s


def config4(seed=4, L_nominal=64.0, n_mesh=49, n_fcc=38):
    """Binary LJ mixture (80:20, sigma 1/0.88, eps 1/0.5, Lorentz-Berthelot) in a
    periodic 64-sigma cube on a jittered 49^3 hex mesh; FCC 38^3 (N=219,488)."""
    L = float(qround(L_nominal))
    nodes = uniform_nodes(L, n_mesh)
    mesh = hex_mesh(nodes, nodes, nodes, periodic_axes=(0, 1, 2))
    mesh = jitter_interior(mesh, nodes, nodes, nodes, 0.25, _rng(seed, 0))
    mesh = renumber_cells(mesh, _rng(seed, 5).permutation(mesh.n_cells))
    a = L / n_fcc
    x = fcc_sites((n_fcc,) * 3, a)
    x = x + _rng(seed, 1).uniform(-0.05, 0.05, size=x.shape)
    lo, hi = np.zeros(3), np.full(3, L)
    x = qround(wrap(qround(x), lo, hi, (0, 1, 2)))
    x = np.where(x >= L, x - L, x)
    N = len(x)
    sp = binary_species(N, 0.8, _rng(seed, 2))
    G = qround(_rng(seed, 4).standard_normal((N, 3)))
    return Workload(f"binary{N}_cube64_mesh{n_mesh}", mesh, x, sp, np.array([1.0, 0.5]),
                    np.array([1.0, 0.88]), 2.5, lo, hi, (0, 1, 2), extra={"G": G, "gamma": 0.1})


def channel_mesh(Lx, Ly, Lz, hx, hy_wall, hy_mid, hz, jitter, rng):
    xs = uniform_nodes(Lx, max(1, int(round(Lx / hx))))
    ys = graded_nodes(Ly, hy_wall, hy_mid)
    zs = uniform_nodes(Lz, max(1, int(round(Lz / hz))))
    mesh = hex_mesh(xs, ys, zs, periodic_axes=(0, 2))
    if jitter > 0:
        mesh = jitter_interior(mesh, xs, ys, zs, jitter, rng)
    return mesh, (xs, ys, zs)


def config5(seed=5, scale=1.0, shuffle=True):
    """400x200x100 channel periodic in x,z with walls in y; graded jittered hex mesh
    of about 4M cells (y spacing 1.0 at the walls to 2.5 at the centre); FCC
    238x119x59 unit cells, N = 6,683,992 (density 0.836).  scale < 1 shrinks
    every length (and N) for smaller tests."""
    Lx, Ly, Lz = (float(qround(v * scale)) for v in (400.0, 200.0, 100.0))
    hxz = 1.07
    mesh, nodes = channel_mesh(Lx, Ly, Lz, hxz, 1.0, 2.5, hxz, 0.25, _rng(seed, 0))
    if shuffle:
        mesh = renumber_cells(mesh, _rng(seed, 5).permutation(mesh.n_cells))
    nf = (max(1, int(round(238 * scale))), max(1, int(round(119 * scale))), max(1, int(round(59 * scale))))
    a = np.array([Lx / nf[0], Ly / nf[1], Lz / nf[2]])
    x = fcc_sites(nf, a)
    x = x + _rng(seed, 1).uniform(-0.05, 0.05, size=x.shape)
    lo, hi = np.zeros(3), np.array([Lx, Ly, Lz])
    x = qround(wrap(qround(x), lo, hi, (0, 2)))
    for ax in (0, 2):
        x[:, ax] = np.where(x[:, ax] >= hi[ax], x[:, ax] - (hi[ax] - lo[ax]), x[:, ax])
    N = len(x)
    return Workload(f"fcc{N}_channel{Lx:g}x{Ly:g}x{Lz:g}_graded", mesh, x, np.zeros(N, np.int32),
                    np.array([1.0]), np.array([1.0]), 2.5, lo, hi, (0, 2), extra={"nodes": nodes})


def small_random(n_mesh=(3, 3, 3), L=(8.0, 8.0, 8.0), N=200, periodic_axes=(0, 1, 2), mesh_jitter=0.25,
                 seed=7, shuffle=True, species_frac=None, min_sep=0.8):
    """Tiny randomized case: jittered hex mesh, random well-separated positions."""
    Ls = [float(qround(v)) for v in L]
    xs, ys, zs = (uniform_nodes(Ls[a], n_mesh[a]) for a in range(3))
    mesh = hex_mesh(xs, ys, zs, periodic_axes=periodic_axes)
    if mesh_jitter > 0:
        mesh = jitter_interior(mesh, xs, ys, zs, mesh_jitter, _rng(seed, 0))
    if shuffle:
        mesh = renumber_cells(mesh, _rng(seed, 5).permutation(mesh.n_cells))
    lo, hi = np.zeros(3), np.array(Ls)
    r = _rng(seed, 1)
    x = lo + r.uniform(0.0, 1.0, size=(N, 3)) * (hi - lo)
    if min_sep > 0:
        x = soft_relax(x, lo, hi, periodic_axes, 100, r0=min_sep, step=0.2, clip=0.1)
    x = qround(x)
    for ax in range(3):
        if ax in periodic_axes:
            x[:, ax] = np.where(x[:, ax] >= hi[ax], x[:, ax] - (hi[ax] - lo[ax]), x[:, ax])
            x[:, ax] = np.where(x[:, ax] < lo[ax], x[:, ax] + (hi[ax] - lo[ax]), x[:, ax])
        else:
            x[:, ax] = np.clip(x[:, ax], lo[ax] + Q, hi[ax] - Q)
    if species_frac is None:
        sp, eps, sig = np.zeros(N, np.int32), np.array([1.0]), np.array([1.0])
    else:
        sp = binary_species(N, species_frac, _rng(seed, 2))
        eps, sig = np.array([1.0, 0.5]), np.array([1.0, 0.88])
    return Workload("small_random", mesh, x, sp, eps, sig, 2.5, lo, hi, tuple(periodic_axes))


def cutoff_band_pairs(n_side=6, spacing=8.0, seed=21):
    """Isolated molecule pairs whose separations d are multiples of Q with |d|^2 within a few FP32
    ulps of rc^2 = 6.25 on both sides (and one pair at exactly rc), on a jittered periodic hex mesh.
    Pairs from different sites are farther apart than rc, so each site holds at most one interacting
    pair; whether it interacts is decided by the exact integer sum a^2 + b^2 + c^2 < (2.5 / Q)^2."""
    rng = _rng(seed, 0)
    R = int(round(2.5 / Q)) ** 2
    L = float(qround(n_side * spacing))
    xi, xj = [], []
    for s in range(n_side ** 3):
        site = np.array([s % n_side, (s // n_side) % n_side, s // n_side ** 2], dtype=np.float64) * spacing
        base = qround(site + rng.uniform(0.5, 1.5, size=3))
        if s == 0:
            abc = np.array([int(round(2.5 / Q)), 0, 0])
        else:
            # aim at R + k; of 256 random (a, b), keep the triple closest to the aim
            k = int(rng.integers(-4000, 4001))
            ab = rng.integers(0, 52000, size=(256, 2)).astype(np.int64)
            rest = R + k - (ab ** 2).sum(1)
            c = np.floor(np.sqrt(rest.astype(np.float64))).astype(np.int64)
            c += ((c + 1) ** 2 <= rest).astype(np.int64) - (c ** 2 > rest).astype(np.int64)
            best = int(np.argmin(rest - c ** 2))
            abc = np.array([ab[best, 0], ab[best, 1], c[best]]) * rng.choice([-1, 1], size=3)
        xi.append(base)
        xj.append(base + abc * Q)
    x = np.vstack([np.array(xi), np.array(xj)])
    x = np.mod(x, L)
    nodes = uniform_nodes(L, 2 * n_side)
    mesh = jitter_interior(hex_mesh(nodes, nodes, nodes, periodic_axes=(0, 1, 2)), nodes, nodes, nodes, 0.2,
                           _rng(seed, 1))
    n = len(x)
    return Workload(f"cutoff_band_{n}", mesh, qround(x), np.zeros(n, np.int32), np.array([1.0]), np.array([1.0]),
                    2.5, np.zeros(3), np.full(3, L), (0, 1, 2))


def refined_nodes(length, centres, half_width, h_fine, h_coarse, slope=0.5):
    """Node coordinates on [0, length]: spacing h_fine within half_width of any centre, growing by
    `slope` per unit distance beyond it, capped at h_coarse (rescaled to end exactly at length)."""
    centres = np.asarray(centres, dtype=np.float64)

    def h(x):
        d = np.min(np.abs(centres - x)) if len(centres) else np.inf
        return min(h_coarse, h_fine + slope * max(0.0, d - half_width))

    xs = [0.0]
    while xs[-1] < length:
        xs.append(xs[-1] + h(xs[-1] + 0.5 * h(xs[-1])))
    xs = np.array(xs)
    if xs[-1] - length > 0.5 * (xs[-1] - xs[-2]):
        xs = xs[:-1]
    return xs * (length / xs[-1])


def config3(seed=3, n_cells_target=6.0e5, post_r=8.0):
    """Nanochannel with posts: 200 x 60 x 60 box, periodic in x and z, walls at y = 0 and 60; six posts
    of radius 8 along z at x_k = 200 (k + 1/2) / 6, y = 30.  Tensor-product hex mesh with spacing 1
    within 12 of a post axis (x) and of y = 30 (y), graded to at most 3 elsewhere, uniform z spacing
    sized for about n_cells_target cells after deleting the cells whose vertices (after a +-0.25 edge
    interior jitter) all lie inside a post.  FCC at density 0.8, sites with r_post >= 8.5 and
    0.5 <= y <= 59.5, jitter +-0.05; Maxwell velocities at T* = 1 with zero net momentum, rescaled
    exactly (extra["v"])."""
    Lx, Ly, Lz = (float(qround(v)) for v in (200.0, 60.0, 60.0))
    posts = np.array([[Lx * (k + 0.5) / 6.0, Ly / 2.0] for k in range(6)])
    xs = refined_nodes(Lx, posts[:, 0], 12.0, 1.0, 3.0)
    ys = refined_nodes(Ly, [Ly / 2.0], 12.0, 1.0, 3.0)
    # cells of the x-y layer outside the posts (cell centres), to size the z spacing
    cxm, cym = np.meshgrid(0.5 * (xs[1:] + xs[:-1]), 0.5 * (ys[1:] + ys[:-1]), indexing="ij")
    rmin = np.min(np.hypot(cxm[..., None] - posts[:, 0], cym[..., None] - posts[:, 1]), axis=-1)
    n_layer = int((rmin >= post_r).sum())
    nz = max(2, int(round(n_cells_target / max(n_layer, 1))))
    zs = uniform_nodes(Lz, nz)
    xs, ys, zs = (qround(a) for a in (xs, ys, zs))
    mesh = hex_mesh(xs, ys, zs, periodic_axes=(0, 2))
    mesh = jitter_interior(mesh, xs, ys, zs, 0.25, _rng(seed, 0))
    # delete the cells whose vertices all lie inside a post (such a cell lies inside the post, which
    # is convex, so every point outside the posts stays in a kept cell)
    pr = np.min(np.hypot(mesh.points[:, 0:1] - posts[:, 0], mesh.points[:, 1:2] - posts[:, 1]), axis=1)
    lens = np.diff(mesh.face_off)
    fmax = np.maximum.reduceat(pr[mesh.face_pts], mesh.face_off[:-1]) if len(lens) else np.zeros(0)
    cmax = np.zeros(mesh.n_cells)
    np.maximum.at(cmax, mesh.owner, fmax)
    nb = mesh.neighbour >= 0
    np.maximum.at(cmax, mesh.neighbour[nb], fmax[nb])
    mesh = delete_cells(mesh, cmax < post_r)
    mesh = renumber_cells(mesh, _rng(seed, 5).permutation(mesh.n_cells))
    # molecules
    a0 = (4.0 / 0.8) ** (1.0 / 3.0)
    nf = (int(round(Lx / a0)), int(round(Ly / a0)), int(round(Lz / a0)))
    a = np.array([Lx / nf[0], Ly / nf[1], Lz / nf[2]])
    x = fcc_sites(nf, a)
    x = x + _rng(seed, 1).uniform(-0.05, 0.05, size=x.shape)
    r = np.min(np.hypot(x[:, 0:1] - posts[:, 0], x[:, 1:2] - posts[:, 1]), axis=1)
    x = x[(r >= post_r + 0.5) & (x[:, 1] >= 0.5) & (x[:, 1] <= Ly - 0.5)]
    lo, hi = np.zeros(3), np.array([Lx, Ly, Lz])
    x = qround(wrap(qround(x), lo, hi, (0, 2)))
    for ax in (0, 2):
        x[:, ax] = np.where(x[:, ax] >= hi[ax], x[:, ax] - (hi[ax] - lo[ax]), x[:, ax])
    N = len(x)
    v = _rng(seed, 3).standard_normal((N, 3))
    v -= v.mean(axis=0)
    v *= np.sqrt(3.0 * N * 1.0 / (v ** 2).sum())
    return Workload(f"posts{N}_channel200x60x60", mesh, x, np.zeros(N, np.int32), np.array([1.0]), np.array([1.0]),
                    2.5, lo, hi, (0, 2), extra={"v": v, "posts": posts, "post_r": post_r})


# ----------------------------------------------------------------------------------------------
# rotationally periodic sector (referring transforms with a rotation, Sec. 2.2.2)


def rot_z(angle):
    """Rotation by `angle` about the z axis."""
    c, s = math.cos(angle), math.sin(angle)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def wedge_mesh(r0, r1, n_sectors, Lz, nr, nphi, nz, jitter, rng, shuffle=True):
    """Hex mesh of one sector (angle 2 pi / n_sectors) of the annulus r0 <= r <= r1, 0 <= z < Lz.

    Nodes at (r_i cos phi_j, r_i sin phi_j, z_k) on a uniform (r, phi, z) grid, interior nodes moved by
    U(-jitter h, jitter h) in (r, phi, z) before the mapping (faces stay planar on the boundary, so the
    sector is bounded by planes through the z axis, chords of the two walls and two z planes).  The
    sides phi = 0 and phi = 2 pi / n_sectors are coupled by the rotation about z, z by the translation
    Lz; the walls r = r0, r1 are plain boundaries."""
    theta = 2.0 * math.pi / n_sectors
    rs = np.linspace(r0, r1, nr + 1)
    ps = np.linspace(0.0, theta, nphi + 1)
    zs = uniform_nodes(Lz, nz)
    m = hex_mesh(rs, ps, zs)
    if jitter > 0:
        m = jitter_interior(m, rs, ps, zs, jitter, rng)
    r, p, z = m.points[:, 0], m.points[:, 1], m.points[:, 2]
    # exact node values on the two coupled sides, so that one is the rotation of the other
    p = np.where(np.isclose(p, 0.0, atol=1e-15), 0.0, p)
    pts = np.stack([r * np.cos(p), r * np.sin(p), z], axis=1)
    side = np.isclose(m.points[:, 1], theta, rtol=0, atol=1e-13)
    pts[side] = (rot_z(theta) @ np.stack([r[side], np.zeros(side.sum()), z[side]], axis=0)).T
    out = Mesh(points=pts, face_off=m.face_off, face_pts=m.face_pts, owner=m.owner, neighbour=m.neighbour,
               n_cells=m.n_cells, periodic=np.array([[0.0, 0.0, 0.0], [0.0, 0.0, Lz]]),
               lo=np.array([0.0, 0.0, 0.0]), hi=np.array([r1, r1, Lz]),
               rotations=np.stack([rot_z(theta), np.eye(3)]))
    out.wedge = dict(r0=r0, r1=r1, n_sectors=n_sectors, theta=theta, Lz=Lz, nr=nr, nphi=nphi, nz=nz)
    if shuffle:
        out2 = renumber_cells(out, rng.permutation(out.n_cells))
        out2.wedge = out.wedge
        out = out2
    return out


def wedge_images(x, n_sectors, Lz, copies=1):
    """Positions of the rotated (powers -copies..copies of the sector rotation) and z-shifted (-1, 0, 1)
    copies of x, with the power pairs: input preparation for minimum-separation checks."""
    theta = 2.0 * math.pi / n_sectors
    out, tags = [], []
    for a in range(-copies, copies + 1):
        Ra = rot_z(a * theta)
        for b in (-1, 0, 1):
            out.append(x @ Ra.T + np.array([0.0, 0.0, b * Lz]))
            tags.append((a, b))
    return out, tags


def wedge_positions(mesh, density, jitter, rng, margin=1e-3):
    """Molecules on rings: z layers and radii at spacing h = density^(-1/3), on each ring
    floor(r theta / h) sites evenly spread over (0, theta), each moved by U(-jitter, jitter) per axis.
    Radii run from r0 + h/2 to the chord of the outer wall less h/2, so every site is inside the mesh;
    sites next to the coupled sides sit half a spacing from them."""
    w = mesh.wedge
    theta, Lz = w["theta"], w["Lz"]
    dphi = theta / w["nphi"]
    h = density ** (-1.0 / 3.0)
    rin, rout = w["r0"] + 0.5 * h, w["r1"] * math.cos(0.5 * dphi) - 0.5 * h
    nrad = int(math.floor((rout - rin) / h)) + 1
    nzl = max(1, int(round(Lz / h)))
    sites = []
    for i in range(nrad):
        r = rin + i * h
        m = max(1, int(math.floor(r * theta / h)))
        p = (np.arange(m) + 0.5) * (theta / m)
        for k in range(nzl):
            z = (k + 0.25 + 0.5 * (i % 2)) * (Lz / nzl)
            sites.append(np.stack([r * np.cos(p), r * np.sin(p), np.full(m, z)], axis=1))
    x = np.vstack(sites)
    x = x + rng.uniform(-jitter, jitter, size=x.shape)
    # stay inside: radial range and the two sides (the jitter is far below h / 2)
    x = qround(x)
    x[:, 2] = np.mod(x[:, 2], Lz)
    return x


def wedge(seed=6, r0=10.0, r1=22.0, n_sectors=12, Lz=8.0, nr=10, nphi=8, nz=6, density=0.7, jitter=0.2):
    """Molecules in a rotationally periodic annular sector (12 sectors of 30 degrees by default), periodic
    in z, walls at r0 and r1; ring-lattice sites at the given density, jittered by +-0.1."""
    rng = _rng(seed, 0)
    mesh = wedge_mesh(r0, r1, n_sectors, qround(Lz), nr, nphi, nz, jitter, rng)
    x = wedge_positions(mesh, density, 0.1, _rng(seed, 1))
    n = len(x)
    return Workload(f"wedge{n}_sector{n_sectors}_r{r0:g}-{r1:g}", mesh, x, np.zeros(n, np.int32), np.array([1.0]),
                    np.array([1.0]), 2.5, mesh.lo, mesh.hi, (), extra={"wedge": mesh.wedge})


def annulus_from_wedge(mesh, x, G=None):
    """The whole annulus: n_sectors rotated copies of the sector mesh (as disjoint cell sets) and of the
    positions (and of per-molecule vectors G), periodic in z only.  Copy s of molecule i is s * N + i."""
    w = mesh.wedge
    K, theta = w["n_sectors"], w["theta"]
    P, F = len(mesh.points), mesh.n_faces
    pts, fo, fp, ow, ne, xs, gs = [], [0], [], [], [], [], []
    for s in range(K):
        Rs = rot_z(s * theta)
        pts.append(mesh.points @ Rs.T)
        fo.extend((mesh.face_off[1:] + fo[-1]).tolist())
        fp.append(mesh.face_pts + s * P)
        ow.append(mesh.owner + s * mesh.n_cells)
        ne.append(np.where(mesh.neighbour >= 0, mesh.neighbour + s * mesh.n_cells, -1))
        xs.append(x @ Rs.T)
        if G is not None:
            gs.append(np.asarray(G) @ Rs.T)
    full = Mesh(points=np.vstack(pts), face_off=np.array(fo, np.int64), face_pts=np.concatenate(fp).astype(np.int32),
                owner=np.concatenate(ow).astype(np.int32), neighbour=np.concatenate(ne).astype(np.int32),
                n_cells=K * mesh.n_cells, periodic=np.array([[0.0, 0.0, w["Lz"]]]))
    return full, np.vstack(xs), (np.vstack(gs) if G is not None else None)
