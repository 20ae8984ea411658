"""Screening census of a workload (TEST/ANALYSIS INFRASTRUCTURE).

Counts, per quartet class (l_a l_b | l_c l_d) in canonical orientation
(l_a >= l_b, l_c >= l_d, bra pair class >= ket pair class), the unique shell
quartets that survive Cauchy-Schwarz screening Q_ab Q_cd >= tau (paper,
section 4.1), the integrals they hold and their primitive quartets.  Schwarz
bounds come from the oracle.

    python -m oracle.census dimer|cluster64|cluster512 [tau]
"""
from __future__ import annotations

import sys

import numpy as np

PAIR_CLASSES = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]
PAIR_NAMES = ["ss", "ps", "pp", "ds", "dp", "dd"]
NC = {0: 1, 1: 3, 2: 6}


def pair_table(mol, Q):
    ls = np.array([s.l for s in mol.shells])
    nps = np.array([len(s.exps) for s in mol.shells])
    i, j = np.tril_indices(mol.nshell)
    la, lb = np.maximum(ls[i], ls[j]), np.minimum(ls[i], ls[j])
    cls = np.array([PAIR_CLASSES.index((a, b)) for a, b in zip(la, lb)], dtype=int)
    return dict(i=i, j=j, cls=cls, q=Q[i, j], kprim=nps[i] * nps[j])


def census(mol, Q, tau):
    pt = pair_table(mol, Q)
    rows = []
    tot = dict(quartets=0, integrals=0, prim=0, unscreened=0)
    for B in range(6):
        qb = pt["q"][pt["cls"] == B]
        kb = pt["kprim"][pt["cls"] == B]
        for K in range(B + 1):
            qk = pt["q"][pt["cls"] == K]
            kk = pt["kprim"][pt["cls"] == K]
            order = np.argsort(-qk)
            qs, ks = qk[order], kk[order]
            kcum = np.concatenate([[0], np.cumsum(ks)])
            with np.errstate(divide="ignore"):
                thr = np.where(qb > 0, tau / np.where(qb > 0, qb, 1), np.inf)
            # number of kets with q >= thr (qs descending)
            cnt = np.searchsorted(-qs, -thr, side="right")
            nq = int(cnt.sum())
            npq = int((kb * kcum[cnt]).sum())
            unscreened = len(qb) * len(qk)
            if B == K:
                diag = qb * qb >= tau
                nq = (nq + int(diag.sum())) // 2
                npq = (npq + int((kb * kb)[diag].sum())) // 2
                unscreened = len(qb) * (len(qb) + 1) // 2
            lb_, lk_ = PAIR_CLASSES[B], PAIR_CLASSES[K]
            nint = nq * NC[lb_[0]] * NC[lb_[1]] * NC[lk_[0]] * NC[lk_[1]]
            rows.append(dict(cls=f"({PAIR_NAMES[B]}|{PAIR_NAMES[K]})", bra_pairs=len(qb), ket_pairs=len(qk),
                             unscreened=unscreened, quartets=nq, integrals=nint, prim_quartets=npq))
            tot["quartets"] += nq
            tot["integrals"] += nint
            tot["prim"] += npq
            tot["unscreened"] += unscreened
    sig = int((pt["q"] * pt["q"].max() >= tau).sum())
    return rows, tot, dict(nshell=mol.nshell, nbf=mol.nbf, pairs=len(pt["q"]), significant_pairs=sig)


def main(argv):
    import workloads as W
    import oracle
    name = argv[1] if len(argv) > 1 else "dimer"
    mol = {"dimer": W.dimer_config, "cluster64": W.cluster64_config,
           "cluster512": W.cluster512_config}[name]()
    tau = float(argv[2]) if len(argv) > 2 else (1e-11 if name == "cluster512" else 1e-10)
    Q = oracle.Basis(mol).schwarz()
    rows, tot, info = census(mol, Q, tau)
    print(f"{name}: {info}, tau={tau}")
    print(f"{'class':12s} {'bra':>9s} {'ket':>9s} {'unscreened':>14s} {'quartets':>14s} {'integrals':>14s} {'prim':>14s}")
    for r in rows:
        print(f"{r['cls']:12s} {r['bra_pairs']:9d} {r['ket_pairs']:9d} {r['unscreened']:14d} {r['quartets']:14d} "
              f"{r['integrals']:14d} {r['prim_quartets']:14d}")
    print(f"total: quartets={tot['quartets']:.4e} integrals={tot['integrals']:.4e} prim={tot['prim']:.4e} "
          f"unscreened={tot['unscreened']:.4e}")


if __name__ == "__main__":
    main(sys.argv)
