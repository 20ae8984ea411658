"""Seeded synthetic workloads: water clusters and their Gaussian basis.

This module is the one input source shared by the HIP library's tests and
the CPU oracle.  It holds geometry and basis *data* only: atom positions,
nuclear charges, shell angular momenta, primitive exponents and the
contraction coefficients of normalised primitives.  It computes nothing of
the Hartree-Fock method (no normalisation, no integrals): each consumer does
its own arithmetic from these raw numbers.

Shapes follow the workloads of the closed-shell Fock build (the paper's
section 5.2 uses graphene bilayers in 6-31G(d); those files are not
available, so seeded water clusters with an even-tempered synthetic basis
stand in for them):

* ``water_dimer(seed)``      -- (H2O)2, O-O 2.9 A, random orientations
                                (26 basis functions without d shells).
* ``water_cluster(n, seed)`` -- n waters on a jittered cubic lattice
                                (3.0 A spacing, +-0.3 A jitter, random
                                orientations); with the d shell on O each
                                water carries 19 basis functions.
* ``cluster_batch(...)``     -- many independent clusters of uneven size.

Units: positions are returned in bohr (1 A = 1/0.529177210903 bohr).
Basis-function order used throughout: atoms in input order, shells in the
order listed per element, Cartesian components lexicographic
(x, y, z) and (xx, xy, xz, yy, yz, zz).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

ANGSTROM_TO_BOHR = 1.0 / 0.529177210903

# Water geometry (Angstrom, degrees).
R_OH = 0.96
THETA_HOH = 104.5
R_OO_DIMER = 2.9
LATTICE_SPACING = 3.0
LATTICE_JITTER = 0.3
CLASH_DISTANCE = 1.5

# The contraction coefficients refer to normalised primitives and are index
# aligned with the exponents (k = 0, 1, 2).
_CONTRACTED_COEFS = (0.15, 0.53, 0.44)


def _even_tempered(base: float, n: int = 3, ratio: float = 3.0) -> tuple:
    return tuple(base * ratio ** k for k in range(n))


# Element -> list of (l, exponents, coefficients).
BASIS_SP = {
    8: [
        (0, _even_tempered(0.2), _CONTRACTED_COEFS),
        (0, (0.3,), (1.0,)),
        (0, (0.08,), (1.0,)),
        (1, (0.8,), (1.0,)),
        (1, (0.2,), (1.0,)),
    ],
    1: [
        (0, _even_tempered(0.15), _CONTRACTED_COEFS),
        (0, (0.12,), (1.0,)),
    ],
}
# Same plus one Cartesian d shell (alpha = 0.8) on oxygen.
BASIS_SPD = {
    8: BASIS_SP[8] + [(2, (0.8,), (1.0,))],
    1: BASIS_SP[1],
}

# Textbook STO-3G hydrogen (Hehre, Stewart, Pople; as tabulated by Szabo and
# Ostlund, section 3.5).  Used for the H2 minimal-basis check.
STO3G_H = {
    1: [
        (0, (3.42525091, 0.62391373, 0.16885540),
         (0.15432897, 0.53532814, 0.44463454)),
    ]
}

# Synthetic carbon basis with the shape of a split-valence basis with one d
# shell (the paper's graphene runs, section 5.2, use 6-31G(d), whose data are
# not available here): a 6-primitive 1s shell, a 3-primitive and a
# 1-primitive SP (L) shell -- s and p sharing exponents, with separate
# coefficients -- and one Cartesian d shell: 4 shells, 15 functions per
# carbon.  Exponents are even-tempered and synthetic; l = -1 marks SP.
SP = -1
BASIS_CARBON = {
    6: [
        (0, tuple(0.9 * 3.4 ** k for k in range(6)), (0.05, 0.20, 0.40, 0.32, 0.13, 0.03)),
        (SP, tuple(0.22 * 3.0 ** k for k in range(3)), (0.45, 0.40, -0.10), (0.30, 0.50, 0.30)),
        (SP, (0.12,), (1.0,), (1.0,)),
        (2, (0.8,), (1.0,)),
    ],
}

NCART = {SP: 4, 0: 1, 1: 3, 2: 6}


@dataclass
class Shell:
    atom: int
    l: int                   # 0, 1, 2, or SP (-1): an s and a p shell sharing exponents
    exps: np.ndarray
    coefs: np.ndarray        # s coefficients for SP
    coefs_p: np.ndarray = None   # SP only: p coefficients

    @property
    def nbf(self) -> int:
        return NCART[self.l]


@dataclass
class Molecule:
    Z: np.ndarray            # (natom,) int32
    xyz: np.ndarray          # (natom, 3) float64, bohr
    shells: List[Shell] = field(default_factory=list)
    name: str = ""

    @property
    def natom(self) -> int:
        return int(self.Z.shape[0])

    @property
    def nshell(self) -> int:
        return len(self.shells)

    @property
    def nbf(self) -> int:
        return sum(s.nbf for s in self.shells)

    @property
    def nelec(self) -> int:
        return int(self.Z.sum())

    @property
    def nocc(self) -> int:
        return self.nelec // 2

    def flat(self) -> dict:
        """Flat arrays (shell table + primitive arrays) for C interfaces."""
        nsh = self.nshell
        sh_atom = np.array([s.atom for s in self.shells], dtype=np.int32)
        sh_l = np.array([s.l for s in self.shells], dtype=np.int32)
        sh_np = np.array([len(s.exps) for s in self.shells], dtype=np.int32)
        sh_off = np.zeros(nsh, dtype=np.int32)
        if nsh:
            sh_off[1:] = np.cumsum(sh_np)[:-1]
        exps = np.concatenate([np.asarray(s.exps, float) for s in self.shells]) if nsh else np.zeros(0)
        coefs = np.concatenate([np.asarray(s.coefs, float) for s in self.shells]) if nsh else np.zeros(0)
        coefs_p = (np.concatenate([np.asarray(s.coefs_p if s.l == SP else np.zeros(len(s.exps)), float)
                                   for s in self.shells]) if nsh else np.zeros(0))
        return dict(natom=self.natom, Z=np.ascontiguousarray(self.Z, dtype=np.int32),
                    xyz=np.ascontiguousarray(self.xyz, dtype=np.float64),
                    nshell=nsh, sh_atom=sh_atom, sh_l=sh_l, sh_np=sh_np, sh_off=sh_off,
                    exps=np.ascontiguousarray(exps), coefs=np.ascontiguousarray(coefs),
                    coefs_p=np.ascontiguousarray(coefs_p))


def attach_basis(Z: Sequence[int], xyz_bohr: np.ndarray, basis: dict, name: str = "") -> Molecule:
    shells = []
    for a, z in enumerate(Z):
        for entry in basis[int(z)]:
            l, ex, co = entry[:3]
            cp = np.array(entry[3], dtype=np.float64) if l == SP else None
            shells.append(Shell(a, l, np.array(ex, dtype=np.float64), np.array(co, dtype=np.float64), cp))
    return Molecule(np.asarray(Z, dtype=np.int32), np.asarray(xyz_bohr, dtype=np.float64), shells, name)


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a unit quaternion of 4 N(0,1) draws."""
    q = rng.standard_normal(4)
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def water_frame() -> np.ndarray:
    """O, H, H positions (Angstrom) of one water in its own frame."""
    half = np.deg2rad(THETA_HOH / 2.0)
    return np.array([
        [0.0, 0.0, 0.0],
        [R_OH * np.sin(half), R_OH * np.cos(half), 0.0],
        [-R_OH * np.sin(half), R_OH * np.cos(half), 0.0],
    ])


def _place_water(o_pos: np.ndarray, rot: np.ndarray) -> np.ndarray:
    return o_pos[None, :] + water_frame() @ rot.T


def water_dimer(seed: int = 0, basis: dict = BASIS_SP) -> Molecule:
    rng = np.random.default_rng(seed)
    atoms = []
    for o_pos in (np.zeros(3), np.array([R_OO_DIMER, 0.0, 0.0])):
        atoms.append(_place_water(o_pos, random_rotation(rng)))
    xyz = np.concatenate(atoms) * ANGSTROM_TO_BOHR
    return attach_basis([8, 1, 1] * 2, xyz, basis, name=f"water_dimer(seed={seed})")


def lattice_sites(n: int) -> np.ndarray:
    """First n sites of the smallest m^3 >= n cubic lattice, nearest the cube
    centre first (ties broken by lexicographic index)."""
    m = 1
    while m ** 3 < n:
        m += 1
    idx = np.array([(i, j, k) for i in range(m) for j in range(m) for k in range(m)], dtype=np.int64)
    pos = idx.astype(np.float64) * LATTICE_SPACING
    centre = (m - 1) / 2.0 * LATTICE_SPACING
    d2 = ((pos - centre) ** 2).sum(axis=1)
    order = sorted(range(len(idx)), key=lambda t: (round(d2[t], 9), tuple(idx[t])))
    return pos[order[:n]]


def water_cluster(n: int, seed: int, basis: dict = BASIS_SPD, return_redraws: bool = False):
    rng = np.random.default_rng(seed)
    sites = lattice_sites(n)
    placed: List[np.ndarray] = []
    redraws = 0
    for s in sites:
        while True:
            o_pos = s + rng.uniform(-LATTICE_JITTER, LATTICE_JITTER, size=3)
            mol = _place_water(o_pos, random_rotation(rng))
            if placed:
                prev = np.concatenate(placed)
                dmin = np.sqrt(((prev[:, None, :] - mol[None, :, :]) ** 2).sum(-1)).min()
                if dmin < CLASH_DISTANCE:
                    redraws += 1
                    continue
            placed.append(mol)
            break
    xyz = np.concatenate(placed) * ANGSTROM_TO_BOHR
    m = attach_basis([8, 1, 1] * n, xyz, basis, name=f"water_cluster(n={n}, seed={seed})")
    return (m, redraws) if return_redraws else m


# Graphene bilayer (section 5.2): two AB-stacked honeycomb layers of carbon,
# C-C 1.42 A, layers 3.35 A apart.
CC_BOND = 1.42
INTERLAYER = 3.35
# atoms per layer of the paper's five systems (Table 4: 44, 120, 220, 356 and
# 2,016 carbon atoms in two layers)
GRAPHENE_SIZES = {"0.5nm": 22, "1nm": 60, "1.5nm": 110, "2nm": 178, "5nm": 1008}


def honeycomb_sites(n: int) -> np.ndarray:
    """The n honeycomb sites (Angstrom, z = 0) nearest the centre of a
    hexagon, ties broken by the lattice indices (i, j, sublattice)."""
    a1 = np.array([1.5 * CC_BOND, np.sqrt(3.0) / 2 * CC_BOND])
    a2 = np.array([1.5 * CC_BOND, -np.sqrt(3.0) / 2 * CC_BOND])
    basis = [np.zeros(2), np.array([CC_BOND, 0.0])]
    centre = np.array([-CC_BOND, 0.0])   # a hexagon centre: distance CC_BOND to its six atoms
    m = 1
    while True:
        cand = []
        for i in range(-m, m + 1):
            for j in range(-m, m + 1):
                for b in range(2):
                    p = i * a1 + j * a2 + basis[b]
                    cand.append((round(float(((p - centre) ** 2).sum()), 9), i, j, b, p))
        cand.sort(key=lambda t: t[:4])
        if len(cand) >= 4 * n and cand[n - 1][0] < (m * CC_BOND) ** 2:
            break
        m += 1
    return np.array([np.append(c[4] - centre, 0.0) for c in cand[:n]])


def graphene_bilayer(n_per_layer: int, basis: dict = BASIS_CARBON) -> Molecule:
    """AB-stacked bilayer flake of 2 n_per_layer carbon atoms: layer 2 is
    layer 1 shifted by one C-C bond in the plane and INTERLAYER along z.
    Deterministic (no random draw)."""
    lay = honeycomb_sites(n_per_layer)
    top = lay + np.array([CC_BOND, 0.0, INTERLAYER])
    xyz = np.concatenate([lay, top]) * ANGSTROM_TO_BOHR
    return attach_basis([6] * (2 * n_per_layer), xyz, basis, name=f"graphene_bilayer({2 * n_per_layer} C)")


def h2(R_bohr: float = 1.4) -> Molecule:
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, R_bohr]])
    return attach_basis([1, 1], xyz, STO3G_H, name=f"H2(R={R_bohr})")


# ---- named workloads ---------------------------------------------------------

def dimer_config() -> Molecule:
    """(H2O)2, seed 0, s/p basis: 18 shells, 26 basis functions."""
    return water_dimer(0, BASIS_SP)


def cluster64_config() -> Molecule:
    """64 waters on a 4^3 jittered lattice, seed 1, s/p/d basis: 1216 BF."""
    return water_cluster(64, 1, BASIS_SPD)


def cluster512_config() -> Molecule:
    """512 waters on an 8^3 jittered lattice, seed 3: 9728 BF."""
    return water_cluster(512, 3, BASIS_SPD)


def batch_sizes(nmol: int = 256, seed: int = 2, lo: int = 1, hi: int = 16) -> np.ndarray:
    return np.random.default_rng(seed).integers(lo, hi + 1, size=nmol)


def cluster_batch(nmol: int = 256, seed: int = 2, lo: int = 1, hi: int = 16,
                  seed_base: int = 2_000_000) -> List[Molecule]:
    """Independent clusters of uneven size: sizes ~ U{lo..hi}; molecule i
    uses seed seed_base + i."""
    sizes = batch_sizes(nmol, seed, lo, hi)
    return [water_cluster(int(n), seed_base + i, BASIS_SPD) for i, n in enumerate(sizes)]


def guess_training_set(count: int = 2000, lo: int = 4, hi: int = 32, size_seed: int = 4,
                       seed_base: int = 10_000) -> List[Molecule]:
    sizes = np.random.default_rng(size_seed).integers(lo, hi + 1, size=count)
    return [water_cluster(int(n), seed_base + i, BASIS_SPD) for i, n in enumerate(sizes)]


def guess_eval_set(count: int = 8, n: int = 128, seed_base: int = 20_000) -> List[Molecule]:
    return [water_cluster(n, seed_base + j, BASIS_SPD) for j in range(count)]


def random_symmetric(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded random symmetric matrix (a test density)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-scale, scale, size=(n, n))
    return 0.5 * (a + a.T)


def random_orthonormal_density(n: int, nocc: int, seed: int) -> np.ndarray:
    """D = C C^T with C an n x nocc matrix of orthonormal columns (a
    projector; idempotent in the Euclidean metric)."""
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, nocc)))
    return q @ q.T
