"""Write tests/golden/c2_energies.json: the two lowest energies of the
24-spinor, 8-electron complex FCI problem (735,471 determinants, integrals
seed 2002) from the oracle's own Davidson on the oracle's Slater-Condon
sigma.  Calls only oracle/ and synth/.  Takes of the order of an hour on a
few CPU cores.

Usage: python tests/golden/make_c2_energies.py [threads]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import csc, davidson, space  # noqa: E402


def main():
    nthreads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    ints, sp, roots = synth.config("c2")
    dets = space.enumerate_dets(sp.n_elec, sp.sub, sp.lo, sp.hi)
    diag = csc.diag(dets, ints.h, ints.g, nthreads=nthreads)
    n_mv = [0]

    def matvec(x):
        n_mv[0] += 1
        return csc.sigma(dets, ints.h, ints.g, x, nthreads=nthreads)

    hist = []
    t0 = time.time()
    tol = 1e-6
    e, X, rn, it = davidson.davidson(matvec, diag, k=roots, tol=tol, max_iter=400, m_max=32, history=hist)
    out = {
        "problem": "complex spinor FCI, 24 spinors, 8 electrons, integrals seed 2002 (rank 32, sigma_f 0.03)",
        "n_dets": int(len(dets)),
        "energies": [float(x) for x in e],
        "resid": [float(x) for x in rn],
        "tol_residual": tol,
        "iterations": int(it),
        "sigma_products": n_mv[0],
        "e1_minus_e0": float(e[1] - e[0]),
        "seconds": round(time.time() - t0, 1),
        "written_by": "tests/golden/make_c2_energies.py (oracle Davidson on the oracle sigma)",
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_energies.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
