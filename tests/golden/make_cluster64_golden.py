"""Write the 64-water full-size fixture from the CPU oracle alone.

Workload: 64 waters on the jittered 4^3 lattice (seed 1), s/p/d basis, 1216
basis functions, Schwarz threshold 1e-10; density D = C C^T with C the
orthonormal columns of a seeded 1216 x 320 Gaussian matrix (seed 21).

The oracle's 8-fold-symmetric build (section 4.1, algorithm 1's loop nest
with the six updates of eq. 2) gives J and K; the fixture keeps what a test
can compare with the GPU build at full size without storing two 1216^2
matrices:

* tr(D J) and tr(D K) (so tr(D (2J - K)), the two-electron energy at fixed D),
* every row sum of J and of K (each element of J and K enters one of them),
* one complete shell block (a, b) for each of the six pair classes
  ss, ps, pp, ds, dp, dd,
* the screened quartet, integral and primitive-quartet counts.

Only ``oracle`` and ``workloads`` are imported.  Runs for about half an hour
on eight cores:

    python tests/golden/make_cluster64_golden.py [OUT.json]
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402

DENSITY_SEED = 21
TAU = 1e-10
# (bra shell, ket shell) per pair class; shells of water w are 10w .. 10w+9
# in the order O s(3), O s, O s, O p, O p, O d, H1 s(3), H1 s, H2 s(3), H2 s.
BLOCKS = {"ss": (0, 6), "ps": (3, 1), "pp": (213, 634), "ds": (5, 318), "dp": (325, 4), "dd": (5, 635)}


def main(out):
    m = W.cluster64_config()
    D = W.random_orthonormal_density(m.nbf, m.nocc, DENSITY_SEED)
    B = oracle.Basis(m)
    t0 = time.time()
    J, K, st = B.jk(D, TAU)
    dt = time.time() - t0
    bf, ls = B.shell_bf, B.shell_l
    blocks = []
    for name, (a, b) in BLOCKS.items():
        la, lb = int(ls[a]), int(ls[b])
        assert "spd"[la] + "spd"[lb] == name, (name, la, lb)
        na, nb = W.NCART[la], W.NCART[lb]
        blocks.append({"pair_class": name, "a": a, "b": b,
                       "J": J[bf[a]:bf[a] + na, bf[b]:bf[b] + nb].tolist(),
                       "K": K[bf[a]:bf[a] + na, bf[b]:bf[b] + nb].tolist()})
    doc = {
        "what": "CPU oracle J and K of the 64-water cluster at a seeded projector density",
        "workload": "workloads.cluster64_config(): 64 waters, seed 1, 640 shells, 1216 basis functions",
        "density": f"workloads.random_orthonormal_density(1216, 320, seed={DENSITY_SEED})",
        "schwarz_tau": TAU,
        "written_by": "tests/golden/make_cluster64_golden.py (calls oracle/ only)",
        "oracle_seconds": round(dt, 1), "oracle_threads": oracle.num_threads(),
        "quartets": st[0], "integrals": st[1], "primitive_quartets": st[2],
        "tr_DJ": float(np.sum(D * J)), "tr_DK": float(np.sum(D * K)),
        "row_sums_J": J.sum(axis=1).tolist(), "row_sums_K": K.sum(axis=1).tolist(),
        "blocks": blocks,
    }
    with open(out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(f"wrote {out}: {st[0]} quartets in {dt:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "cluster64_oracle_jk.json"))
