"""MI355X-native AICA Lennard-Jones pair forces (arXiv cs/0702131), Python binding.

The functions below carry the C ABI's names and only marshal arguments: mesh
arrays go in as host NumPy arrays, positions and results are torch device
tensors, and every computation runs in the HIP library (libaica.so).  The
library must be built (``__graft_entry__.build()``); there is no CPU path.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (AICA_E_INVAL, AICA_E_MESH, AICA_E_RCUT, AICA_E_UNLOCATED, AICA_FP32, AICA_FP64, AicaError,
                   aica_info, aica_mesh, aica_params, check, lib)

__all__ = ["DIL", "aica_build_dil", "aica_bin", "aica_forces", "aica_forces_noalloc", "aica_forces_adjoint", "aica_pairs_export",
           "aica_pair_counts",
           "aica_dil_export", "aica_bin_export", "AicaLJ", "AicaError", "AICA_FP32", "AICA_FP64",
           "AICA_E_INVAL", "AICA_E_MESH", "AICA_E_RCUT", "AICA_E_UNLOCATED"]


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class DIL:
    """Owns an aica_dil handle: the mesh's interaction lists and the per-step binning state."""

    def __init__(self, mesh, rcut, guard=None, predicate="closest"):
        """predicate "closest" (default): cell pairs whose closest points are within rcut + guard;
        "vertex": the paper's vertex-to-vertex test, which can miss pairs on distorted meshes."""
        self.rcut = float(rcut)
        self.guard = 1e-6 * self.rcut if guard is None else float(guard)
        pts = _c(mesh.points, np.float64)
        fo = _c(mesh.face_off, np.int64)
        fp = _c(mesh.face_pts, np.int32)
        ow = _c(mesh.owner, np.int32)
        ne = _c(mesh.neighbour, np.int32)
        per = np.asarray(mesh.periodic, dtype=np.float64).reshape(-1, 3)
        m = aica_mesh()
        m.n_points, m.points = len(pts), pts.ctypes.data
        m.n_faces, m.face_off, m.face_pts = len(ow), fo.ctypes.data, fp.ctypes.data
        m.owner, m.neighbour, m.n_cells = ow.ctypes.data, ne.ctypes.data, int(mesh.n_cells)
        m.n_periodic = len(per)
        for k in range(len(per)):
            for q in range(3):
                m.periodic_vec[k][q] = per[k, q]
        rot = getattr(mesh, "rotations", None)
        if rot is not None:  # referring transforms x -> R_k x + y_k (kept alive until the call returns)
            rot = np.ascontiguousarray(np.asarray(rot, dtype=np.float64).reshape(len(per), 3, 3))
            m.periodic_rot = rot.ctypes.data
        h = C.c_void_p()
        pred = {"closest": _lib.AICA_DIL_CLOSEST, "vertex": _lib.AICA_DIL_VERTEX}[predicate]
        check(lib().aica_build_dil_ex(C.byref(m), self.rcut, self.guard, pred, C.byref(h)))
        self.h = h
        self.n_cells = int(mesh.n_cells)
        self._pos = None

    def close(self):
        if getattr(self, "h", None):
            lib().aica_dil_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        inf = aica_info()
        check(lib().aica_dil_info(self.h, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in aica_info._fields_}

    def work_stats(self):
        """(DIL candidate pairs of the last binning, lane-pair evaluations executed by the last forward call)."""
        a, b = C.c_int64(), C.c_int64()
        check(lib().aica_work_stats(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def profile(self, enable=True):
        check(lib().aica_profile(self.h, 1 if enable else 0))

    def profile_read(self, kernel, reset=True):
        ms, n = C.c_double(), C.c_int64()
        check(lib().aica_profile_read(self.h, kernel.encode(), C.byref(ms), C.byref(n), 1 if reset else 0))
        return ms.value, n.value


def aica_build_dil(mesh, rcut, guard=None, predicate="closest"):
    return DIL(mesh, rcut, guard, predicate)


def _stream(t):
    import torch
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return AICA_FP64
    if t.dtype == torch.float32:
        return AICA_FP32
    raise TypeError("positions must be float32 or float64")


def _check_pos(pos):
    if not pos.is_cuda or pos.dim() != 2 or pos.shape[1] != 3 or not pos.is_contiguous():
        raise ValueError("positions must be a contiguous [n, 3] device tensor")


def aica_bin(dil: DIL, pos):
    """Locate every molecule's cell and build the CSR occupancy (keeps pos alive in the handle)."""
    _check_pos(pos)
    check(lib().aica_bin(dil.h, C.c_void_p(pos.data_ptr()), _dtype_code(pos), pos.shape[0], _stream(pos)))
    dil._pos = pos


def _params(rcut, eps, sigma, precision, compensated):
    eps = _c(np.atleast_1d(np.asarray(eps, dtype=np.float64)), np.float64)
    sig = _c(np.atleast_1d(np.asarray(sigma, dtype=np.float64)), np.float64)
    # the library reads n_species entries of both arrays
    if eps.ndim != 1 or sig.shape != eps.shape:
        raise ValueError("eps and sigma must be 1-D with one entry per species each")
    p = aica_params()
    p.rcut = float(rcut)
    p.n_species = len(eps)
    p.eps, p.sigma = eps.ctypes.data, sig.ctypes.data
    p.precision = AICA_FP32 if precision in ("fp32", AICA_FP32) else AICA_FP64
    p.compensated = 1 if compensated else 0
    return p, (eps, sig)


def _species_ptr(species, pos):
    if species is None:
        return C.c_void_p(0)
    import torch
    if (species.dtype != torch.int32 or not species.is_cuda or species.device != pos.device
            or species.dim() != 1 or species.shape[0] != pos.shape[0] or not species.is_contiguous()):
        raise ValueError("species must be a contiguous int32 tensor of length n on the positions' device")
    return C.c_void_p(species.data_ptr())


def _check_grad_forces(grad_forces, pos):
    """The upstream gradient G must be an [n, 3] tensor on the positions' device (a host tensor would hand
    the kernels a host pointer; fewer rows would be read past their end)."""
    if (not hasattr(grad_forces, "is_cuda") or not grad_forces.is_cuda or grad_forces.device != pos.device
            or grad_forces.dim() != 2 or tuple(grad_forces.shape) != (pos.shape[0], 3)):
        raise ValueError("grad_forces must be an [n, 3] tensor on the positions' device")


def aica_forces(dil: DIL, pos, species=None, eps=(1.0,), sigma=(1.0,), rcut=None, precision="fp32",
                compensated=True):
    """Forces [n,3] (caller order, compute dtype), uw = [U, W] (float64) and npairs (int64), on device."""
    import torch
    _check_pos(pos)
    p, keep = _params(dil.rcut if rcut is None else rcut, eps, sigma, precision, compensated)
    dt = torch.float32 if p.precision == AICA_FP32 else torch.float64
    F = torch.empty((pos.shape[0], 3), dtype=dt, device=pos.device)
    uw = torch.empty(2, dtype=torch.float64, device=pos.device)
    npairs = torch.empty(1, dtype=torch.int64, device=pos.device)
    check(lib().aica_forces(dil.h, C.c_void_p(pos.data_ptr()), _species_ptr(species, pos), C.byref(p),
                            C.c_void_p(F.data_ptr()), C.c_void_p(uw.data_ptr()), C.c_void_p(npairs.data_ptr()),
                            _stream(pos)))
    return F, uw, npairs


def aica_forces_noalloc(dil: DIL, pos, species=None, eps=(1.0,), sigma=(1.0,), rcut=None, precision="fp32",
                        compensated=True, out=None):
    """As aica_forces, with every device buffer of the call in the library's fixed scratch array (nothing is
    allocated by the library).  out = (F, uw, npairs) preallocated by the caller, or None to allocate them here."""
    import torch
    _check_pos(pos)
    p, keep = _params(dil.rcut if rcut is None else rcut, eps, sigma, precision, compensated)
    dt = torch.float32 if p.precision == AICA_FP32 else torch.float64
    if out is None:
        out = (torch.empty((pos.shape[0], 3), dtype=dt, device=pos.device),
               torch.empty(2, dtype=torch.float64, device=pos.device),
               torch.empty(1, dtype=torch.int64, device=pos.device))
    F, uw, npairs = out
    for t, shape, want in ((F, (pos.shape[0], 3), dt), (uw, (2,), torch.float64), (npairs, (1,), torch.int64)):
        if tuple(t.shape) != shape or t.dtype != want or t.device != pos.device or not t.is_contiguous():
            raise ValueError(f"output tensor must be contiguous {want} of shape {shape} on {pos.device}")
    check(lib().aica_forces_noalloc(dil.h, C.c_void_p(pos.data_ptr()), _species_ptr(species, pos), C.byref(p),
                                    C.c_void_p(F.data_ptr()), C.c_void_p(uw.data_ptr()),
                                    C.c_void_p(npairs.data_ptr()), _stream(pos)))
    return F, uw, npairs


def aica_forces_adjoint(dil: DIL, pos, grad_forces, grad_energy, species=None, eps=(1.0,), sigma=(1.0,),
                        rcut=None, precision="fp32"):
    """dL/dx [n,3], dL/deps [n_species], dL/dsigma [n_species] for L = sum G.F + gamma U."""
    import torch
    _check_pos(pos)
    _check_grad_forces(grad_forces, pos)
    p, keep = _params(dil.rcut if rcut is None else rcut, eps, sigma, precision, True)
    dt = torch.float32 if p.precision == AICA_FP32 else torch.float64
    G = grad_forces.to(dtype=dt).contiguous()
    gx = torch.empty((pos.shape[0], 3), dtype=dt, device=pos.device)
    ge = torch.empty(p.n_species, dtype=torch.float64, device=pos.device)
    gs = torch.empty(p.n_species, dtype=torch.float64, device=pos.device)
    check(lib().aica_forces_adjoint(dil.h, C.c_void_p(pos.data_ptr()), _species_ptr(species, pos), C.byref(p),
                                    C.c_void_p(G.data_ptr()), float(grad_energy), C.c_void_p(gx.data_ptr()),
                                    C.c_void_p(ge.data_ptr()), C.c_void_p(gs.data_ptr()), _stream(pos)))
    return gx, ge, gs


def aica_pairs_export(dil: DIL, pos, rcut=None, precision="fp32"):
    """The pairs the GPU path finds inside the cut-off, canonical (a, b, n0, n1, n2) rows, sorted."""
    _check_pos(pos)
    p, keep = _params(dil.rcut if rcut is None else rcut, (1.0,), (1.0,), precision, False)
    cap = max(1024, 64 * pos.shape[0])
    while True:
        a = np.zeros(cap, np.int32)
        b = np.zeros(cap, np.int32)
        im = np.zeros((cap, 3), np.int8)
        n = C.c_int64()
        check(lib().aica_pairs_export(dil.h, C.c_void_p(pos.data_ptr()), C.byref(p), cap, C.byref(n),
                                      a.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p),
                                      im.ctypes.data_as(C.c_void_p), _stream(pos)))
        if n.value <= cap:
            break
        cap = n.value
    k = n.value
    key = np.stack([a[:k], b[:k], im[:k, 0], im[:k, 1], im[:k, 2]], axis=1).astype(np.int64)
    return key[np.lexsort(key.T[::-1])]


def aica_pair_counts(dil: DIL, pos, rcut=None, precision="fp32"):
    """Pairs inside the cut-off per molecule ([n] int32 on the device, caller order), from the traversal of
    aica_forces."""
    import torch
    _check_pos(pos)
    p, keep = _params(dil.rcut if rcut is None else rcut, (1.0,), (1.0,), precision, False)
    counts = torch.empty(pos.shape[0], dtype=torch.int32, device=pos.device)
    check(lib().aica_pair_counts(dil.h, C.c_void_p(pos.data_ptr()), C.byref(p), C.c_void_p(counts.data_ptr()),
                                 _stream(pos)))
    return counts


def aica_dil_export(dil: DIL):
    """Interacting cell pairs (c, d, n0, n1, n2) in mesh cell ids, sorted."""
    n = C.c_int64()
    check(lib().aica_dil_export(dil.h, C.byref(n), None, None, None))
    k = n.value
    c = np.zeros(k, np.int32)
    d = np.zeros(k, np.int32)
    im = np.zeros((k, 3), np.int8)
    check(lib().aica_dil_export(dil.h, C.byref(n), c.ctypes.data_as(C.c_void_p), d.ctypes.data_as(C.c_void_p),
                                im.ctypes.data_as(C.c_void_p)))
    key = np.stack([c, d, im[:, 0], im[:, 1], im[:, 2]], axis=1).astype(np.int64)
    return key[np.lexsort(key.T[::-1])]


def aica_bin_export(dil: DIL, n):
    cell_of = np.zeros(n, np.int32)
    order = np.zeros(n, np.int32)
    count = np.zeros(dil.n_cells, np.int64)
    check(lib().aica_bin_export(dil.h, cell_of.ctypes.data_as(C.c_void_p), order.ctypes.data_as(C.c_void_p),
                                count.ctypes.data_as(C.c_void_p)))
    return cell_of, order, count


from .autograd import AicaLJ  # noqa: E402
