"""CPU FP64 oracle of the learned initial guess (test infrastructure only).

Not part of the product path: tests, the smoke check and the benchmark's CPU
leg are its only callers.

The learned guess is one of the extensions of the closed-shell SCF (the
paper starts SCF from a core-Hamiltonian path, section 3; the network is not
in the paper).  What it computes, in this module's plain form:

* atom pairs (A, B) within 6 A (A = B included), ordered O before H, then by
  atom index; pair type 0 = O-O, 1 = O-H, 2 = H-H;
* a 164-number descriptor per pair: one-hot elements of A and B, 32 radial
  Gaussians of R_AB with a cosine cutoff, and each atom's environment
  (log(1 + the same radial functions summed over its neighbours), per
  element: the logarithm keeps highly coordinated atoms near the range of
  the small training clusters);
* a right-handed local frame per pair (z from A to B; x toward the nearest
  non-collinear neighbour of A) and the matrices that rotate Cartesian
  s, p and unit-normalised d functions into it;
* the density block of the pair in that frame, P = T_A^-T D_AB T_B^-1, so
  that D_AB = T_A^T P T_B;
* a multilayer perceptron (164 -> 256 -> 256 -> 256 with SiLU, then one
  linear head per pair type: 225, 30 or 4 outputs = the block) on inputs
  standardised with the stored mean and scale and clipped to +-4, trained
  with the mean squared error and Adam.

Parity of every function here is pinned by tests of its own: the rotation
matrices against direct evaluation of the rotated functions, frame
covariance of the local blocks under rigid motions, the descriptor's
invariance, the analytic gradient against central finite differences and
Adam against its closed-form first step.
"""
from __future__ import annotations

import numpy as np

BOHR_PER_ANGSTROM = 1.0 / 0.529177210903
ELEMENTS = (8, 1)                       # one-hot order
NRAD = 32
RCUT_A = 6.0
MU_A = np.linspace(0.5, 6.0, NRAD)
DMU_A = MU_A[1] - MU_A[0]
ETA_A = 1.0 / (2.0 * DMU_A ** 2)
NFEAT = 2 + 2 + NRAD + 2 * 2 * NRAD     # 164
HIDDEN = 256
NLAYER = 3
NTYPE = 3
# distance ties (equal O-H bonds) are broken by atom index below this
TIE_BOHR = 1e-6
NONCOLLINEAR_SIN = 0.1
INPUT_CLIP = 4.0


def element_index(z: int) -> int:
    return ELEMENTS.index(int(z))


def cutoff(r_a: float) -> float:
    return 0.5 * (np.cos(np.pi * r_a / RCUT_A) + 1.0) if r_a < RCUT_A else 0.0


def radial(r_a: float) -> np.ndarray:
    """G_k(r) = exp(-eta (r - mu_k)^2) f_c(r), r in Angstrom."""
    return np.exp(-ETA_A * (r_a - MU_A) ** 2) * cutoff(r_a)


def atom_functions(mol):
    """Per atom: (first basis function, list of shell l) in basis order."""
    first = {}
    ls = {a: [] for a in range(mol.natom)}
    off = 0
    for s in mol.shells:
        first.setdefault(s.atom, off)
        ls[s.atom].append(s.l)
        off += s.nbf
    return [first.get(a, 0) for a in range(mol.natom)], [ls[a] for a in range(mol.natom)]


def pair_type(za: int, zb: int) -> int:
    return element_index(za) + element_index(zb)     # OO 0, OH 1, HH 2


def pair_list(mol):
    """[(A, B, type)] for R_AB < 6 A and A <= B in the element-then-index order."""
    out = []
    n = mol.natom
    for a in range(n):
        for b in range(n):
            ea, eb = element_index(mol.Z[a]), element_index(mol.Z[b])
            if (ea, a) > (eb, b):
                continue                              # O first, then lower index
            r = np.linalg.norm(mol.xyz[a] - mol.xyz[b]) / BOHR_PER_ANGSTROM
            if r < RCUT_A:
                out.append((a, b, pair_type(mol.Z[a], mol.Z[b])))
    out.sort(key=lambda p: (p[2], p[0], p[1]))
    return out


def features(mol, pairs) -> np.ndarray:
    """(npair, 164) descriptors: [onehot A, onehot B, G(R_AB), env_A, env_B],
    env_X = log(1 + sum over atoms C != X of G(R_XC)), one 32-block per
    element of C."""
    n = mol.natom
    env = np.zeros((n, 2 * NRAD))
    for x in range(n):
        for c in range(n):
            if c == x:
                continue
            r = np.linalg.norm(mol.xyz[x] - mol.xyz[c]) / BOHR_PER_ANGSTROM
            e = element_index(mol.Z[c])
            env[x, e * NRAD:(e + 1) * NRAD] += radial(r)
    env = np.log1p(env)
    X = np.zeros((len(pairs), NFEAT))
    for i, (a, b, _) in enumerate(pairs):
        X[i, element_index(mol.Z[a])] = 1.0
        X[i, 2 + element_index(mol.Z[b])] = 1.0
        r = np.linalg.norm(mol.xyz[a] - mol.xyz[b]) / BOHR_PER_ANGSTROM
        X[i, 4:4 + NRAD] = radial(r)
        X[i, 4 + NRAD:4 + 3 * NRAD] = env[a]
        X[i, 4 + 3 * NRAD:] = env[b]
    return X


def _by_distance(mol, a, exclude):
    cands = [c for c in range(mol.natom) if c not in exclude]
    key = lambda c: (np.floor(np.linalg.norm(mol.xyz[c] - mol.xyz[a]) / TIE_BOHR), c)
    return sorted(cands, key=key)


def frame(mol, a: int, b: int) -> np.ndarray:
    """Rows = local x, y, z axes in global coordinates (local r' = R r).

    z points from A to B; for A = B it points from A to A's nearest atom.
    x is the part of (C - A) normal to z for the nearest atom C (distance, then
    index) not collinear with z (sine above 0.1); without one, the global
    axis least aligned with z (lowest index on ties).  y = z x x."""
    if a == b:
        near = _by_distance(mol, a, {a})
        if not near:
            return np.eye(3)
        b = near[0]
    z = mol.xyz[b] - mol.xyz[a]
    z = z / np.linalg.norm(z)
    x = None
    for c in _by_distance(mol, a, {a, b}):
        v = mol.xyz[c] - mol.xyz[a]
        u = v / np.linalg.norm(v)
        if np.linalg.norm(np.cross(u, z)) > NONCOLLINEAR_SIN:
            x = v - np.dot(v, z) * z
            break
    if x is None:
        k = int(np.argmin(np.abs(z)))
        e = np.zeros(3)
        e[k] = 1.0
        x = e - np.dot(e, z) * z
    x = x / np.linalg.norm(x)
    y = np.cross(z, x)
    return np.array([x, y, z])


D_COMPONENTS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))
D_NORM = np.array([1 / np.sqrt(3.0), 1.0, 1.0, 1 / np.sqrt(3.0), 1.0, 1 / np.sqrt(3.0)])


def cart_transform(l: int, R: np.ndarray) -> np.ndarray:
    """T with phi(R r) = T phi(r) for the unit-normalised Cartesian shell l
    (components in the order x, y, z and xx, xy, xz, yy, yz, zz)."""
    if l == 0:
        return np.ones((1, 1))
    if l == 1:
        return R.copy()
    M = np.zeros((6, 6))
    for p, (a, b) in enumerate(D_COMPONENTS):
        for q, (i, j) in enumerate(D_COMPONENTS):
            M[p, q] = R[a, i] * R[b, j] + (R[a, j] * R[b, i] if i != j else 0.0)
    return np.diag(D_NORM) @ M @ np.diag(1.0 / D_NORM)


def atom_transform(shell_ls, R) -> np.ndarray:
    blocks = [cart_transform(l, R) for l in shell_ls]
    n = sum(b.shape[0] for b in blocks)
    T = np.zeros((n, n))
    o = 0
    for b in blocks:
        k = b.shape[0]
        T[o:o + k, o:o + k] = b
        o += k
    return T


def block_sizes(mol):
    _, ls = atom_functions(mol)
    return [sum((1, 3, 6)[l] for l in x) for x in ls]


def local_blocks(mol, pairs, D) -> list:
    """P_AB = T_A^-T D_AB T_B^-1 in each pair's frame (T^-1 = T(R^T))."""
    first, ls = atom_functions(mol)
    nb = block_sizes(mol)
    out = []
    for a, b, _ in pairs:
        R = frame(mol, a, b)
        Tai = atom_transform(ls[a], R.T)
        Tbi = atom_transform(ls[b], R.T)
        Dab = D[first[a]:first[a] + nb[a], first[b]:first[b] + nb[b]]
        out.append(Tai.T @ Dab @ Tbi)
    return out


def assemble(mol, pairs, blocks, D_base) -> np.ndarray:
    """D = D_base + sum over pairs of T_A^T P T_B placed at (A, B) and its
    transpose at (B, A); a self block uses (P + P^T) / 2."""
    first, ls = atom_functions(mol)
    nb = block_sizes(mol)
    D = np.array(D_base, dtype=float, copy=True)
    for (a, b, _), P in zip(pairs, blocks):
        R = frame(mol, a, b)
        P = np.asarray(P, float).reshape(nb[a], nb[b])
        if a == b:
            P = 0.5 * (P + P.T)
        G = atom_transform(ls[a], R).T @ P @ atom_transform(ls[b], R)
        D[first[a]:first[a] + nb[a], first[b]:first[b] + nb[b]] += G
        if a != b:
            D[first[b]:first[b] + nb[b], first[a]:first[a] + nb[a]] += G.T
    return D


# ---- the network -----------------------------------------------------------------------

HEAD_OUT = (225, 30, 4)


def param_shapes():
    """Packed FP32 parameter layout shared with the library's model format:
    W1 b1 W2 b2 W3 b3, then per head W b, then feature mean, feature scale
    and the three target scales (W is out x in, row-major)."""
    shapes = [("W1", (HIDDEN, NFEAT)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
              ("W3", (HIDDEN, HIDDEN)), ("b3", (HIDDEN,))]
    for t, n in enumerate(HEAD_OUT):
        shapes += [(f"H{t}", (n, HIDDEN)), (f"c{t}", (n,))]
    shapes += [("fmean", (NFEAT,)), ("fscale", (NFEAT,)), ("tscale", (NTYPE,))]
    return shapes


TRAINABLE = 12      # the first 12 arrays are weights and biases


def unpack(flat):
    out, o = {}, 0
    for name, shp in param_shapes():
        n = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + n], dtype=float).reshape(shp)
        o += n
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], float).ravel() for name, _ in param_shapes()])


def param_count() -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes())


def init_params(seed: int, fmean=None, fscale=None, tscale=None):
    """He-style uniform initialisation (seeded); heads start at zero so the
    untrained network predicts the SAD density."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in param_shapes():
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shp[1])
            p[name] = rng.uniform(-lim, lim, size=shp)
        elif name.startswith("H"):
            lim = np.sqrt(6.0 / shp[1]) * 0.1
            p[name] = rng.uniform(-lim, lim, size=shp)
        else:
            p[name] = np.zeros(shp)
    p["fmean"] = np.zeros(NFEAT) if fmean is None else np.asarray(fmean, float)
    p["fscale"] = np.ones(NFEAT) if fscale is None else np.asarray(fscale, float)
    p["tscale"] = np.ones(NTYPE) if tscale is None else np.asarray(tscale, float)
    return p


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, X, counts, keep=False):
    """Rows of X are grouped by pair type (counts[t] rows of type t).
    Returns the scaled outputs per type [Y_t] (block = Y_t * tscale[t])."""
    h = np.clip((np.asarray(X, float) - p["fmean"]) / p["fscale"], -INPUT_CLIP, INPUT_CLIP)
    hs, zs = [h], []
    for k in (1, 2, 3):
        z = hs[-1] @ p[f"W{k}"].T + p[f"b{k}"]
        zs.append(z)
        hs.append(silu(z))
    Ys, o = [], 0
    for t in range(NTYPE):
        Ys.append(hs[-1][o:o + counts[t]] @ p[f"H{t}"].T + p[f"c{t}"])
        o += counts[t]
    return (Ys, hs, zs) if keep else Ys


def predict_blocks(p, X, counts):
    return [Y * p["tscale"][t] for t, Y in enumerate(forward(p, X, counts))]


def loss_and_grad(p, X, counts, T):
    """Mean squared error between Y_t and T_t / tscale[t] over every element
    of every type; returns (loss, grads dict for the trainable arrays)."""
    Ys, hs, zs = forward(p, X, counts, keep=True)
    total = sum(Y.size for Y in Ys)
    loss = 0.0
    g = {}
    dh = np.zeros_like(hs[-1])
    o = 0
    for t in range(NTYPE):
        d = Ys[t] - np.asarray(T[t], float) / p["tscale"][t]
        loss += float(np.sum(d * d))
        dY = 2.0 * d / total
        g[f"H{t}"] = dY.T @ hs[-1][o:o + counts[t]]
        g[f"c{t}"] = dY.sum(0)
        dh[o:o + counts[t]] = dY @ p[f"H{t}"]
        o += counts[t]
    for k in (3, 2, 1):
        dz = dh * dsilu(zs[k - 1])
        g[f"W{k}"] = dz.T @ hs[k - 1]
        g[f"b{k}"] = dz.sum(0)
        dh = dz @ p[f"W{k}"]
    return loss / total, g


def adam(p, g, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba) on the trainable arrays, in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for name, _ in param_shapes()[:TRAINABLE]:
        m = state.setdefault("m_" + name, np.zeros_like(p[name]))
        v = state.setdefault("v_" + name, np.zeros_like(p[name]))
        m[...] = b1 * m + (1 - b1) * g[name]
        v[...] = b2 * v + (1 - b2) * g[name] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[name] = p[name] - lr * mh / (np.sqrt(vh) + eps)
    return p
