"""Write the stored FP64 oracle results of the binary-mixture differentiation case.

Workload: the 80:20 Lennard-Jones mixture of 219,488 molecules in the periodic 64-sigma cube on the
jittered 49^3 hex mesh (sigma_A 1, sigma_B 0.88, eps_A 1, eps_B 0.5, Lorentz-Berthelot, rc 2.5), with
L = sum_a G_a . F_a + gamma U, G ~ N(0, 1) rounded to multiples of 2^-15 and gamma = 0.1.

Everything here comes from the CPU oracle (all pairs, all images, FP64):
  - L, dL/deps_s and dL/dsigma_s from the analytic adjoint;
  - central finite differences of L in each of (eps_A, eps_B, sigma_A, sigma_B) with h = 1e-6 (eight
    full evaluations of L; the cut-off is absolute, so the pair set does not move with the parameters);
  - dL/dx on 1,024 rows drawn with a fixed seed, and the rms of dL/dx over every molecule.

Run from the repository root (about 2-3 hours on 8 cores):
    OMP_NUM_THREADS=8 python tests/golden/make_binary_adjoint.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "binary219488_adjoint.txt")
H = 1e-6
NROWS = 1024
ROW_SEED = 0xAD70


def sample_rows(n):
    """The fixed rows at which dL/dx is stored (sorted)."""
    return np.sort(np.random.default_rng(ROW_SEED).choice(n, NROWS, replace=False))


def read(path=OUT):
    """The stored results: a dict of the scalar lines (floats, or float arrays for the per-species pairs)
    plus 'rows' (int64 [NROWS]) and 'dLdx' (float64 [NROWS, 3])."""
    out, rows, vals = {}, [], []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            f = line.split()
            if f[0][0].isdigit():
                rows.append(int(f[0]))
                vals.append([float(v) for v in f[1:4]])
            elif len(f) == 2:
                out[f[0]] = float(f[1])
            else:
                out[f[0]] = np.array([float(v) for v in f[1:]])
    out["rows"] = np.array(rows, dtype=np.int64)
    out["dLdx"] = np.array(vals, dtype=np.float64)
    return out


def main():
    from oracle import oracle as O
    from paper_cs_0702131_amd import workloads as W

    t0 = time.time()
    wl = W.config4()
    G, gamma = wl.extra["G"], wl.extra["gamma"]
    per = wl.mesh.periodic
    print(f"{wl.name}: {wl.n} molecules", flush=True)
    gx, ge, gs, L = O.adjoint(wl.x, wl.species, wl.eps, wl.sigma, wl.rcut, per, G, gamma)
    print(f"adjoint done ({time.time() - t0:.0f} s): L = {L!r}", flush=True)
    rows = sample_rows(wl.n)
    rms = float(np.sqrt(np.mean(gx ** 2)))
    fd = []
    for which, base in (("eps", wl.eps), ("sigma", wl.sigma)):
        for s in range(len(base)):
            vals = []
            for sign in (1.0, -1.0):
                p = np.array(base, dtype=np.float64)
                p[s] += sign * H
                eps, sig = (p, wl.sigma) if which == "eps" else (wl.eps, p)
                vals.append(O.loss(wl.x, wl.species, eps, sig, wl.rcut, per, G, gamma))
                print(f"  L({which}_{s} {'+' if sign > 0 else '-'} h) = {vals[-1]!r} ({time.time() - t0:.0f} s)",
                      flush=True)
            fd.append((vals[0] - vals[1]) / (2 * H))
    with open(OUT + ".tmp", "w") as fh:
        fh.write("# Binary Lennard-Jones mixture, 219,488 molecules, periodic 64-sigma cube, 49^3 jittered hex mesh\n")
        fh.write("# (80:20 A:B, sigma 1/0.88, eps 1/0.5, Lorentz-Berthelot, rc 2.5 absolute);\n")
        fh.write("# L = sum_a G_a . F_a + gamma U with G ~ N(0,1) rounded to 2^-15, gamma = 0.1.\n")
        fh.write("# FP64 CPU oracle (all pairs, all images); written by tests/golden/make_binary_adjoint.py.\n")
        fh.write(f"n {wl.n}\n")
        fh.write(f"L {float(L)!r}\n")
        fh.write(f"grad_eps {float(ge[0])!r} {float(ge[1])!r}\n")
        fh.write(f"grad_sigma {float(gs[0])!r} {float(gs[1])!r}\n")
        fh.write(f"fd_h {H!r}\n")
        fh.write(f"fd_eps {float(fd[0])!r} {float(fd[1])!r}\n")
        fh.write(f"fd_sigma {float(fd[2])!r} {float(fd[3])!r}\n")
        fh.write(f"rms_dLdx_all {rms!r}\n")
        fh.write(f"row_seed {ROW_SEED}\n")
        fh.write("# row  dL/dx  dL/dy  dL/dz\n")
        for r in rows:
            fh.write(f"{r} {float(gx[r, 0])!r} {float(gx[r, 1])!r} {float(gx[r, 2])!r}\n")
    os.replace(OUT + ".tmp", OUT)
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
