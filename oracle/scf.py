"""Plain numpy closed-shell RHF driver for the oracle (TEST INFRASTRUCTURE).

Section 3 of the paper: solve F C = S C eps (eq. 1) by self-consistent
field iterations: core Hamiltonian and initial density, orthogonalisation,
diagonalise, rebuild the density, repeat until consecutive densities agree.
Conventions (shared with the library by specification, not by code):

* D = C_occ C_occ^T (no factor 2), F = H + 2J - K, E = tr(D (H + F)) + E_nuc.
* Orthogonaliser: X = S^{-1/2} (symmetric) when every eigenvalue of S is
  >= ``lindep``; otherwise canonical X = U_k s_k^{-1/2} over the kept
  eigenvectors.
* Pulay DIIS on e = X^T (F D S - S D F) X, at most ``diis_max`` vectors,
  oldest dropped first; extrapolation starts once two vectors are stored.
* Converged when |E_k - E_{k-1}| < e_tol and rms(D_{k+1} - D_k) < d_tol.
* SAD guess: for each element, a spherically averaged fractional-occupation
  atomic RHF in that element's own basis (electron pairs spread evenly over
  the degenerate orbitals at the Fermi level, degeneracy window 1e-4 Eh);
  the molecular guess is the block-diagonal superposition.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import Basis


def orthogonaliser(S: np.ndarray, lindep: float = 1e-7):
    s, U = np.linalg.eigh(S)
    if s.min() >= lindep:
        return (U * s ** -0.5) @ U.T, 0
    keep = s >= lindep
    return U[:, keep] * s[keep] ** -0.5, int((~keep).sum())


def fractional_occupation(eps: np.ndarray, npairs: float, window: float = 1e-4) -> np.ndarray:
    order = np.argsort(eps, kind="stable")
    occ = np.zeros(len(eps))
    remaining = float(npairs)
    i = 0
    while remaining > 1e-14 and i < len(order):
        j = i
        while j + 1 < len(order) and eps[order[j + 1]] - eps[order[i]] < window:
            j += 1
        g = j - i + 1
        if remaining >= g - 1e-14:
            occ[order[i:j + 1]] = 1.0
            remaining -= g
        else:
            occ[order[i:j + 1]] = remaining / g
            remaining = 0.0
        i = j + 1
    return occ


class Diis:
    def __init__(self, nmax: int = 8):
        self.nmax = nmax
        self.F: List[np.ndarray] = []
        self.e: List[np.ndarray] = []

    def push(self, F, e):
        self.F.append(F.copy())
        self.e.append(e.copy())
        if len(self.F) > self.nmax:
            self.F.pop(0)
            self.e.pop(0)

    def extrapolate(self, F):
        while len(self.F) >= 2:
            m = len(self.F)
            B = np.zeros((m + 1, m + 1))
            for i in range(m):
                for j in range(m):
                    B[i, j] = np.vdot(self.e[i], self.e[j])
            B[:m, m] = B[m, :m] = -1.0
            rhs = np.zeros(m + 1)
            rhs[m] = -1.0
            if np.linalg.cond(B) > 1e14:
                self.F.pop(0)
                self.e.pop(0)
                continue
            c = np.linalg.solve(B, rhs)[:m]
            return sum(ci * Fi for ci, Fi in zip(c, self.F))
        return F


@dataclass
class ScfResult:
    energy: float
    e_nuc: float
    iterations: int
    converged: bool
    D: np.ndarray
    C: np.ndarray
    eps: np.ndarray
    history: List[float] = field(default_factory=list)
    ndropped: int = 0


def _density(F, X, nocc):
    eps, Cp = np.linalg.eigh(X.T @ F @ X)
    C = X @ Cp
    return C[:, :nocc] @ C[:, :nocc].T, C, eps


def atomic_density(z: int, basis_shells, tau: float = 0.0, max_iter: int = 200) -> np.ndarray:
    """Spherically averaged fractional-occupation atomic RHF density for one
    element in its own basis (the SAD building block)."""
    import workloads as W
    mol = W.Molecule(np.array([z], dtype=np.int32), np.zeros((1, 3)),
                     [W.Shell(0, s.l, s.exps, s.coefs, getattr(s, "coefs_p", None)) for s in basis_shells])
    B = Basis(mol)
    S, T, V, _ = B.one_electron()
    H = T + V
    X, _ = orthogonaliser(S)
    npairs = z / 2.0
    eps, Cp = np.linalg.eigh(X.T @ H @ X)
    C = X @ Cp
    occ = fractional_occupation(eps, npairs)
    D = (C * occ) @ C.T
    e_old = None
    diis = Diis(8)
    for _ in range(max_iter):
        F = H + B.fock_2e(D, tau)
        E = float(np.sum(D * (H + F)))
        err = X.T @ (F @ D @ S - S @ D @ F) @ X
        diis.push(F, err)
        Fx = diis.extrapolate(F)
        eps, Cp = np.linalg.eigh(X.T @ Fx @ X)
        C = X @ Cp
        occ = fractional_occupation(eps, npairs)
        Dn = (C * occ) @ C.T
        dD = np.sqrt(np.mean((Dn - D) ** 2))
        D = Dn
        if e_old is not None and abs(E - e_old) < 1e-11 and dD < 1e-9:
            break
        e_old = E
    return D


def sad_guess(mol, tau: float = 0.0) -> np.ndarray:
    cache: Dict[int, np.ndarray] = {}
    blocks = []
    for a, z in enumerate(mol.Z):
        shells = [s for s in mol.shells if s.atom == a]
        key = int(z)
        if key not in cache:
            cache[key] = atomic_density(key, shells, tau)
        blocks.append(cache[key])
    n = mol.nbf
    D = np.zeros((n, n))
    o = 0
    for blk in blocks:
        k = blk.shape[0]
        D[o:o + k, o:o + k] = blk
        o += k
    return D


def rhf(mol, tau: float = 1e-10, e_tol: float = 1e-8, d_tol: float = 1e-7, max_iter: int = 100,
        diis_max: int = 8, guess: str = "sad", D0: Optional[np.ndarray] = None,
        lindep: float = 1e-7) -> ScfResult:
    B = Basis(mol)
    S, T, V, enuc = B.one_electron()
    H = T + V
    X, ndrop = orthogonaliser(S, lindep)
    nocc = mol.nocc
    if D0 is not None:
        D = np.array(D0, dtype=np.float64)
    elif guess == "core":
        D, _, _ = _density(H, X, nocc)
    else:
        D = sad_guess(mol)
    diis = Diis(diis_max)
    e_old = None
    hist = []
    C = eps = None
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        F = H + B.fock_2e(D, tau)
        E = float(np.sum(D * (H + F))) + enuc
        hist.append(E)
        err = X.T @ (F @ D @ S - S @ D @ F) @ X
        diis.push(F, err)
        Fx = diis.extrapolate(F)
        Dn, C, eps = _density(Fx, X, nocc)
        dD = np.sqrt(np.mean((Dn - D) ** 2))
        D = Dn
        if e_old is not None and abs(E - e_old) < e_tol and dD < d_tol:
            converged = True
            break
        e_old = E
    return ScfResult(hist[-1], enuc, it, converged, D, C, eps, hist, ndrop)
