#!/usr/bin/env python3
"""Writes the stored reference of the EA-ADC(3) O=20, V=180, Naux=600 system
(the seeded 8-root workload): its lowest 8 eigenvalues and spectroscopic
factors (Eq. 50) from the CPU oracle alone -- the spin-adapted DF sigma of
oracle.radc and the textbook block Davidson of oracle.davidson (block 16,
diagonal preconditioner, residual norms <= 1e-3 Eh absolute, i.e. 1e-9 of
the |omega| ~ 1e6 Eh roots, and eigenvalue changes <= 1e-8 Eh).  Nothing
here calls the HIP library.

Usage: python tests/golden/make_ea_adc3_o20v180.py  (about an hour on 8 cores)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle.davidson import davidson  # noqa: E402
from oracle.radc import RADC  # noqa: E402
from synthetic import make_system  # noqa: E402

OUT = os.path.join(HERE, "ea_adc3_o20v180_roots.json")


def main():
    eps, B, wl = make_system("c2")
    t0 = time.time()
    ref = RADC(eps, B, wl.nocc, wl.order, wl.kind, lazy=True)
    diag = ref.diag()
    print(f"setup + diagonal {time.time() - t0:.1f} s, dim {ref.dim}", flush=True)
    nsig = [0]

    def sigma(X):
        nsig[0] += X.shape[0]
        t = time.time()
        out = ref.sigma(X)
        print(f"  sigma on {X.shape[0]} vectors: {time.time() - t:.1f} s "
              f"({nsig[0]} so far)", flush=True)
        return out

    log = []
    e, X, it, conv = davidson(sigma, diag, wl.nroots, block=wl.block, tol_e=1e-8, tol_r=1e-3,
                              max_iter=200, log=log)
    P = ref.spec_factors(X)
    res = np.linalg.norm(ref.sigma(X) - e[:, None] * X, axis=1)
    rec = {
        "system": "ea-adc3-o20v180 (EA-ADC(3), nocc 20, nvir 180, naux 600, seed 2012069140)",
        "method": "oracle.radc.RADC sigma + oracle.davidson.davidson, block 16, "
                  "tol_e 1e-8 Eh, tol_r 1e-3 Eh",
        "converged": bool(conv), "iterations": int(it), "sigma_vectors": int(nsig[0]),
        "energies_Eh": [float(x) for x in e],
        "spec_factors": [float(x) for x in P],
        "residual_norms_Eh": [float(x) for x in res],
        "seconds": time.time() - t0,
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
