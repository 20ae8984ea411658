"""Pins of the learned-guess oracle against facts that do not come from it:
direct evaluation of rotated Cartesian functions, rigid-motion covariance of
converged SCF densities, descriptor closed forms and invariance, central
finite differences of the loss and the closed-form first Adam step."""
import numpy as np
import pytest

import workloads as W
from oracle import guess as G


def _rotation(seed):
    q = np.random.default_rng(seed).normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


def _moved(mol, Q, t):
    return W.Molecule(mol.Z.copy(), mol.xyz @ Q.T + t, mol.shells, mol.name + " moved")


def _cart_values(l, r):
    """Angular factors of the unit-normalised Cartesian shell at point r
    (the common radial factor and normalisation dropped)."""
    x, y, z = r
    if l == 1:
        return np.array([x, y, z])
    s3 = 1 / np.sqrt(3.0)
    return np.array([s3 * x * x, x * y, x * z, s3 * y * y, y * z, s3 * z * z])


@pytest.mark.parametrize("l", [1, 2])
def test_cart_transform_matches_rotated_functions(l):
    rng = np.random.default_rng(l)
    for seed in range(3):
        R = _rotation(100 + seed)
        T = G.cart_transform(l, R)
        for _ in range(5):
            r = rng.normal(size=3)
            assert np.allclose(_cart_values(l, R @ r), T @ _cart_values(l, r), atol=1e-13)


def test_frames_orthonormal_and_oriented():
    m = W.water_cluster(3, 8)
    for a, b, _ in G.pair_list(m):
        R = G.frame(m, a, b)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(R) - 1.0) < 1e-13
        if a != b:
            v = m.xyz[b] - m.xyz[a]
            assert np.allclose(R[2], v / np.linalg.norm(v), atol=1e-13)


def test_pair_list_and_descriptor_closed_form():
    # two hydrogens 1 A apart: one H-H pair plus two self pairs
    m = W.Molecule(np.array([1, 1], np.int32), np.array([[0, 0, 0], [0, 0, 1.0 * G.BOHR_PER_ANGSTROM]]),
                   [W.Shell(0, 0, np.array([1.0]), np.array([1.0])), W.Shell(1, 0, np.array([1.0]), np.array([1.0]))])
    pairs = G.pair_list(m)
    assert pairs == [(0, 0, 2), (0, 1, 2), (1, 1, 2)]
    X = G.features(m, pairs)
    g1 = np.exp(-G.ETA_A * (1.0 - G.MU_A) ** 2) * 0.5 * (np.cos(np.pi / 6.0) + 1.0)
    g0 = np.exp(-G.ETA_A * G.MU_A ** 2)
    assert X.shape == (3, 164)
    assert np.allclose(X[1, :4], [0, 1, 0, 1])
    assert np.allclose(X[1, 4:36], g1) and np.allclose(X[0, 4:36], g0)
    assert np.allclose(X[1, 36 + 32:36 + 64], np.log1p(g1)) and np.allclose(X[1, 36:68], 0.0)   # A's H neighbour
    # beyond the cutoff: no pair, no environment
    m.xyz[1, 2] = 6.5 * G.BOHR_PER_ANGSTROM
    assert G.pair_list(m) == [(0, 0, 2), (1, 1, 2)]
    assert np.allclose(G.features(m, G.pair_list(m))[:, 36:], 0.0)


def test_descriptor_invariance():
    m = W.water_cluster(4, 12)
    moved = _moved(m, _rotation(5), np.array([1.0, -2.0, 0.5]))
    p0, p1 = G.pair_list(m), G.pair_list(moved)
    assert p0 == p1
    assert np.allclose(G.features(m, p0), G.features(moved, p1), atol=1e-12)
    assert sum(1 for a, b, _ in p0 if a == b) == m.natom
    assert len(p0) == len(set((a, b) for a, b, _ in p0))


def test_local_blocks_covariant_with_converged_density():
    """SCF densities of a rotated and translated molecule, taken into the
    pair frames, agree block by block (frames and p/d transforms)."""
    from oracle import scf
    m = W.water_cluster(2, 17)
    Q = _rotation(9)
    moved = _moved(m, Q, np.array([0.7, 0.1, -1.3]))
    r0 = scf.rhf(m, tau=0.0, e_tol=1e-11, d_tol=1e-9)
    r1 = scf.rhf(moved, tau=0.0, e_tol=1e-11, d_tol=1e-9)
    assert abs(r0.energy - r1.energy) < 1e-9
    pairs = G.pair_list(m)
    b0 = G.local_blocks(m, pairs, r0.D)
    b1 = G.local_blocks(moved, pairs, r1.D)
    for x, y in zip(b0, b1):
        assert np.abs(x - y).max() < 1e-6
    # the global blocks themselves are not invariant (p and d rotate)
    first, _ = G.atom_functions(m)
    assert np.abs(r0.D[first[0]:first[0] + 15, first[0]:first[0] + 15]
                  - r1.D[first[0]:first[0] + 15, first[0]:first[0] + 15]).max() > 1e-3


def test_assemble_inverts_local_blocks():
    m = W.water_cluster(3, 4)
    D = W.random_symmetric(m.nbf, 3, 0.5)
    pairs = G.pair_list(m)
    blocks = G.local_blocks(m, pairs, D)
    back = G.assemble(m, pairs, blocks, np.zeros_like(D))
    first, _ = G.atom_functions(m)
    nb = G.block_sizes(m)
    for a, b, _ in pairs:
        sa = slice(first[a], first[a] + nb[a])
        sb = slice(first[b], first[b] + nb[b])
        assert np.allclose(back[sa, sb], D[sa, sb], atol=1e-12)
        assert np.allclose(back[sb, sa], D[sb, sa], atol=1e-12)


def _small_problem(seed=0):
    rng = np.random.default_rng(seed)
    counts = [3, 4, 2]
    X = rng.normal(size=(sum(counts), G.NFEAT))
    p = G.init_params(seed, fmean=rng.normal(size=G.NFEAT) * 0.1, fscale=rng.uniform(0.5, 2, G.NFEAT),
                      tscale=np.array([0.1, 0.05, 0.02]))
    for t, n in enumerate(G.HEAD_OUT):     # non-zero heads so every path carries gradient
        p[f"H{t}"] = rng.normal(size=(n, G.HIDDEN)) * 0.05
        p[f"c{t}"] = rng.normal(size=n) * 0.01
    T = [rng.normal(size=(c, n)) * 0.03 for c, n in zip(counts, G.HEAD_OUT)]
    return p, X, counts, T


def test_silu_derivative():
    z = np.linspace(-6, 6, 41)
    h = 1e-6
    assert np.allclose(G.dsilu(z), (G.silu(z + h) - G.silu(z - h)) / (2 * h), rtol=1e-8, atol=1e-10)


def test_gradient_matches_finite_differences():
    p, X, counts, T = _small_problem(1)
    _, g = G.loss_and_grad(p, X, counts, T)
    rng = np.random.default_rng(2)
    h = 1e-5
    for name, shp in G.param_shapes()[:G.TRAINABLE]:
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in shp)
            q = {k: v.copy() for k, v in p.items()}
            q[name][idx] += h
            lp, _ = G.loss_and_grad(q, X, counts, T)
            q[name][idx] -= 2 * h
            lm, _ = G.loss_and_grad(q, X, counts, T)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(abs(fd), 1e-6), (name, idx, fd, g[name][idx])


def test_adam_first_step_closed_form():
    p, X, counts, T = _small_problem(3)
    _, g = G.loss_and_grad(p, X, counts, T)
    q = {k: v.copy() for k, v in p.items()}
    G.adam(q, g, {}, lr=1e-3)
    for name, _ in G.param_shapes()[:G.TRAINABLE]:
        # m_hat = g, v_hat = g^2 on step 1
        assert np.allclose(q[name], p[name] - 1e-3 * g[name] / (np.abs(g[name]) + 1e-8), atol=1e-15)


def test_training_reduces_loss():
    p, X, counts, T = _small_problem(4)
    st = {}
    l0, _ = G.loss_and_grad(p, X, counts, T)
    for _ in range(30):
        _, g = G.loss_and_grad(p, X, counts, T)
        G.adam(p, g, st, lr=1e-3)
    l1, _ = G.loss_and_grad(p, X, counts, T)
    assert l1 < 0.5 * l0


def test_inputs_clipped():
    """Standardised inputs beyond +-4 act as +-4: the output is unchanged
    when an input is pushed further out."""
    p, X, counts, _ = _small_problem(6)
    X = X.copy()
    X[0, 10] = p["fmean"][10] + 5.0 * p["fscale"][10]
    Y0 = G.forward(p, X, counts)
    X[0, 10] = p["fmean"][10] + 50.0 * p["fscale"][10]
    Y1 = G.forward(p, X, counts)
    assert all(np.array_equal(a, b) for a, b in zip(Y0, Y1))


def test_pack_roundtrip():
    p, _, _, _ = _small_problem(5)
    flat = G.pack(p)
    assert flat.size == G.param_count()
    q = G.unpack(flat)
    for k in p:
        assert np.array_equal(p[k], q[k])
