#!/usr/bin/env python3
"""Write ``converged_nk8_o8_v24.json``: the oracle's converged CCSD solution of the 2x2x2-mesh
(N_k = 8) system with n_occ = 8, n_vir = 24 spin orbitals per k.

Inputs: the seeded synthetic recipe (seed 202, complex Gaussians x 0.05/N_k, antisymmetrized
and Hermitized, diagonal Fock).  Iteration: the update t <- t + D^-1 R of Sec. 4.4 from
t = 0 (whose first step gives the start t0 = f(0) of Sec. 3.2.2), Pulay DIIS(6), until the
2-norm of (R1, R2) is below 1e-12.  Stored: the complex correlation energy, the iteration
count and norm history, t1 in full, and a fingerprint of t2 (its 2-norm and 512 elements at
seeded positions).  This script calls only ``oracle/`` and ``synth/``; running it takes
about 20 minutes on 8 cores.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import ccsd_k as O  # noqa: E402

GRID, NO, NV, SEED = (2, 2, 2), 8, 24, 202
N = 8
SCALE = 0.05 / N
TOL = 1e-12
NSAMPLE = 512


def sample_positions(kc):
    """NSAMPLE positions (ki, kj, ka, i, j, a, b) drawn from a fixed numpy generator."""
    rng = np.random.default_rng(20191100242)
    pos = []
    for _ in range(NSAMPLE):
        ki, kj, ka = (int(x) for x in rng.integers(0, N, 3))
        i, j = (int(x) for x in rng.integers(0, NO, 2))
        a, b = (int(x) for x in rng.integers(0, NV, 2))
        pos.append([ki, kj, ka, i, j, a, b])
    return pos


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "converged_nk8_o8_v24.json")
    f, eris = synth.system(SEED, GRID, NO, NV, scale=SCALE)
    t0 = time.time()

    def log(it, rn, e):
        print(f"iter {it:3d}  |R| {rn:.3e}  E {e.real:.12f} {e.imag:+.3e}  ({time.time() - t0:.0f} s)", flush=True)

    ref = O.solve(f, eris, GRID, max_iter=60, tol=TOL, diis_space=6, callback=log)
    assert ref["converged"], "oracle did not converge"
    kc = O.kconserv(GRID)
    pos = sample_positions(kc)
    t2 = ref["t2"]
    vals = [t2[tuple(p)] for p in pos]
    rec = dict(
        what="oracle converged CCSD, 2x2x2 mesh, n_occ 8, n_vir 24, seed 202, scale 0.05/8, DIIS(6), tol 1e-12",
        grid=list(GRID), n_occ=NO, n_vir=NV, seed=SEED, eri_scale=SCALE, diis_space=6, tol=TOL,
        iterations=ref["iterations"], rnorm=ref["rnorm"],
        history=[[int(it), float(rn)] for (it, rn, _) in ref["history"]],
        energy=[ref["energy"].real, ref["energy"].imag],
        t2_norm=float(np.linalg.norm(t2.ravel())),
        t1=[[float(x.real), float(x.imag)] for x in ref["t1"].ravel()],
        t2_positions=pos,
        t2_values=[[float(v.real), float(v.imag)] for v in vals],
    )
    with open(out, "w") as fh:
        json.dump(rec, fh, separators=(",", ":"))
    print("wrote", out)


if __name__ == "__main__":
    main()
