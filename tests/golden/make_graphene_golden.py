"""Write the graphene-bilayer SCF fixture from the CPU oracle alone.

Workload: workloads.graphene_bilayer(4) -- an AB-stacked bilayer of 2 x 4
carbon atoms (the shape of the paper's graphene systems, section 5.2, at a
size the oracle converges in about a minute), synthetic split-valence basis
with SP shells and a d shell (4 shells, 15 functions per carbon: 120 basis
functions), Schwarz threshold 1e-10.  The oracle's closed-shell SCF
(section 3, eq. 1; SAD start, DIIS) is converged (|dE| < 1e-10, rms dD < 1e-8) and its energy,
iteration count and Tr(D S) are stored.

    python tests/golden/make_graphene_golden.py [OUT.json]
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from oracle import scf  # noqa: E402


def main(out):
    m = W.graphene_bilayer(4)
    t0 = time.time()
    r = scf.rhf(m, tau=1e-10, e_tol=1e-10, d_tol=1e-8)
    dt = time.time() - t0
    S = oracle.Basis(m).one_electron()[0]
    doc = {"what": "CPU oracle RHF energy of an 8-carbon graphene bilayer with SP shells",
           "workload": "workloads.graphene_bilayer(4): 8 C, 32 shells (SP counted once), 120 basis functions",
           "schwarz_tau": 1e-10, "e_tol": 1e-10, "d_rms_tol": 1e-8,
           "written_by": "tests/golden/make_graphene_golden.py (calls oracle/ only)",
           "converged": bool(r.converged), "iterations": len(r.history), "energy": r.energy,
           "trace_DS": float(np.sum(r.D * S)), "nocc": m.nocc, "oracle_seconds": round(dt, 1)}
    with open(out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(f"wrote {out}: E = {r.energy:.12f} ({len(r.history)} iterations, {dt:.0f} s)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "graphene8_oracle_scf.json"))
