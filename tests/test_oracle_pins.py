"""Pins for the CPU oracle: each check ties it to something other than
itself (a library routine, a textbook value, a brute-force quadrature, a
finite difference, an invariance), so that a dropped term, a wrong sign or
a transposed index in the oracle fails here."""
import json
import os

import numpy as np
import pytest
from scipy import special

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---- Boys function ------------------------------------------------------------

def boys_incomplete_gamma(m, T):
    """F_m(T) = Gamma(m+1/2) P(m+1/2, T) / (2 T^{m+1/2}) (regularised lower
    incomplete gamma, scipy)."""
    if T == 0.0:
        return 1.0 / (2 * m + 1)
    a = m + 0.5
    return special.gamma(a) * special.gammainc(a, T) / (2.0 * T ** a)


@pytest.mark.parametrize("T", [0.0, 1e-12, 1e-6, 0.05, 0.7, 3.3, 9.99, 17.0, 29.999, 30.0, 36.5, 60.0, 120.0, 200.0])
def test_boys_vs_incomplete_gamma(oracle_lib, T):
    F = oracle_lib.boys(16, T)
    for m in range(17):
        ref = boys_incomplete_gamma(m, T)
        assert abs(F[m] - ref) <= 1e-13 * abs(ref) + 1e-300, (m, T, F[m], ref)


def test_boys_zero_and_recursion(oracle_lib):
    F0 = oracle_lib.boys(12, 0.0)
    assert np.allclose(F0, 1.0 / (2 * np.arange(13) + 1), rtol=1e-15, atol=0)
    for T in (0.3, 4.0, 25.0, 45.0):
        F = oracle_lib.boys(12, T)
        for m in range(12):   # downward identity F_m = (2T F_{m+1} + e^-T) / (2m+1)
            assert abs(F[m] - (2 * T * F[m + 1] + np.exp(-T)) / (2 * m + 1)) <= 1e-13 * F[m]


# ---- H2 / STO-3G textbook values ------------------------------------------------

def _h2_with_ghost(R):
    """H2 where the second nucleus carries no charge (its basis stays): V then
    holds nucleus 1's attraction alone."""
    m = W.h2(R)
    m.Z = np.array([1, 0], dtype=np.int32)
    return m


def test_h2_textbook(oracle_lib):
    import oracle
    from oracle import scf
    g = json.load(open(os.path.join(GOLDEN, "h2_sto3g_szabo_ostlund.json")))
    v, tol = g["values"], g["tolerance"]
    m = W.h2(g["R_bohr"])
    B = oracle.Basis(m)
    S, T, V, enuc = B.one_electron()
    _, _, V1, _ = oracle.Basis(_h2_with_ghost(g["R_bohr"])).one_electron()
    eri = B.eri_full()
    H = T + V
    checks = {
        "S12": S[0, 1], "T11": T[0, 0], "T12": T[0, 1],
        "V11_nucleus1": V1[0, 0], "V12_nucleus1": V1[0, 1], "V22_nucleus1": V1[1, 1],
        "H11": H[0, 0], "H12": H[0, 1],
        "eri_11_11": eri[0, 0, 0, 0], "eri_11_22": eri[0, 0, 1, 1],
        "eri_21_21": eri[1, 0, 1, 0], "eri_21_11": eri[1, 0, 0, 0],
    }
    for k, val in checks.items():
        assert abs(val - v[k]) < tol, (k, val, v[k])
    r = scf.rhf(m, tau=0.0, e_tol=1e-12, d_tol=1e-10, guess="core")
    assert r.converged
    assert abs(r.energy - v["E_total"]) < tol
    assert abs(r.energy - enuc - v["E_elec"]) < tol
    # symmetry fixes the closed-shell solution: sigma_g = (1 + 2)/sqrt(2(1+S12))
    s12 = S[0, 1]
    hgg = (H[0, 0] + H[0, 1]) / (1 + s12)
    jgg = (eri[0, 0, 0, 0] + eri[0, 0, 1, 1] + 2 * eri[0, 1, 0, 1] + 4 * eri[0, 0, 0, 1]) / (2 * (1 + s12) ** 2)
    assert abs(r.energy - (2 * hgg + jgg + 1.0 / g["R_bohr"])) < 1e-12


# ---- s-type ERIs against a 3-D quadrature -----------------------------------------

def _gauss_hermite_3d(n, centre, expo):
    x, w = np.polynomial.hermite.hermgauss(n)
    s = 1.0 / np.sqrt(expo)
    g = x * s
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    WW = (w[:, None, None] * w[None, :, None] * w[None, None, :]) * s ** 3
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1) + centre
    base = np.exp(-expo * ((pts - centre) ** 2).sum(1))
    return pts, WW.ravel() / base


def _norm_s(a):
    return (2 * a / np.pi) ** 0.75


def test_ssss_against_quadrature(oracle_lib):
    """(ab|cd) = int rho_ab(r) V_cd(r) d^3r with rho_ab the plain product of
    the two normalised Gaussians on a Gauss-Hermite grid and V_cd the
    potential of the Gaussian charge rho_cd (Gauss's law: the potential of a
    normalised spherical Gaussian of exponent q is erf(sqrt(q) r)/r)."""
    import oracle
    rng = np.random.default_rng(7)
    for trial in range(4):
        ex = rng.uniform(0.15, 2.0, size=4)
        cen = rng.uniform(-1.2, 1.2, size=(4, 3))
        shells = [W.Shell(i, 0, np.array([ex[i]]), np.array([1.0])) for i in range(4)]
        m = W.Molecule(np.zeros(4, dtype=np.int32), cen, shells)
        val = oracle.Basis(m).eri_shell(0, 1, 2, 3)[0, 0, 0, 0]
        a, b, c, d = ex
        A, B, Cc, D = cen
        q = c + d
        Q = (c * Cc + d * D) / q
        qtot = _norm_s(c) * _norm_s(d) * np.exp(-c * d / q * ((Cc - D) ** 2).sum()) * (np.pi / q) ** 1.5
        p = a + b
        P = (a * A + b * B) / p
        pts, w = _gauss_hermite_3d(48, P, p)
        rho = _norm_s(a) * _norm_s(b) * np.exp(-a * ((pts - A) ** 2).sum(1) - b * ((pts - B) ** 2).sum(1))
        r = np.sqrt(((pts - Q) ** 2).sum(1))
        pot = qtot * np.where(r > 1e-12, special.erf(np.sqrt(q) * r) / np.maximum(r, 1e-300), 2 * np.sqrt(q / np.pi))
        quad = float((w * rho * pot).sum())
        assert abs(val - quad) < 1e-10 * abs(quad), (trial, val, quad)


def test_overlap_kinetic_against_quadrature(oracle_lib):
    """S and T for s, p, d primitives on a Gauss-Hermite grid (the Laplacian
    of the ket applied analytically to the plain polynomial*Gaussian)."""
    import oracle
    rng = np.random.default_rng(11)
    ex = [0.6, 1.1]
    cen = rng.uniform(-0.8, 0.8, size=(2, 3))
    for la in range(3):
        for lb in range(3):
            shells = [W.Shell(0, la, np.array([ex[0]]), np.array([1.0])),
                      W.Shell(1, lb, np.array([ex[1]]), np.array([1.0]))]
            m = W.Molecule(np.zeros(2, dtype=np.int32), cen, shells)
            S, T, _, _ = oracle.Basis(m).one_electron()
            na = W.NCART[la]
            p = sum(ex)
            P = (ex[0] * cen[0] + ex[1] * cen[1]) / p
            pts, w = _gauss_hermite_3d(30, P, p)

            def comps(l):
                return [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]

            def dfo(n):
                return np.prod(np.arange(2 * n - 1, 0, -2)) if n > 0 else 1.0

            def val(l, k, a, A, deriv=False):
                lx = comps(l)[k]
                norm = (2 * a / np.pi) ** 0.75 * (4 * a) ** (l / 2) / np.sqrt(dfo(lx[0]) * dfo(lx[1]) * dfo(lx[2]))
                d = pts - A
                g = np.exp(-a * (d ** 2).sum(1))
                poly = d[:, 0] ** lx[0] * d[:, 1] ** lx[1] * d[:, 2] ** lx[2]
                if not deriv:
                    return norm * poly * g
                lap = 0.0
                for ax in range(3):
                    n_ = lx[ax]
                    o = [d[:, i] ** lx[i] for i in range(3)]
                    rest = np.prod([o[i] for i in range(3) if i != ax], axis=0)
                    t = (n_ * (n_ - 1) * d[:, ax] ** max(n_ - 2, 0) if n_ >= 2 else 0.0) \
                        - 2 * a * (2 * n_ + 1) * d[:, ax] ** n_ + 4 * a * a * d[:, ax] ** (n_ + 2)
                    lap = lap + t * rest
                return norm * lap * g

            for i in range(na):
                for j in range(W.NCART[lb]):
                    fa = val(la, i, ex[0], cen[0])
                    s_q = (w * fa * val(lb, j, ex[1], cen[1])).sum()
                    t_q = -0.5 * (w * fa * val(lb, j, ex[1], cen[1], deriv=True)).sum()
                    assert abs(S[i, na + j] - s_q) < 1e-11, (la, lb, i, j)
                    assert abs(T[i, na + j] - t_q) < 1e-10, (la, lb, i, j)
            assert np.allclose(np.diag(S), 1.0, atol=1e-13)


# ---- p and d ERIs against finite differences in the centres ------------------------

def _prim_mol(ls, ex, cen):
    shells = [W.Shell(i, l, np.array([e]), np.array([1.0])) for i, (l, e) in enumerate(zip(ls, ex))]
    return W.Molecule(np.zeros(len(ls), dtype=np.int32), np.array(cen, dtype=float), shells)


def _richardson(f, h):
    d1 = (f(h) - f(-h)) / (2 * h)
    d2 = (f(h / 2) - f(-h / 2)) / h
    return (4 * d2 - d1) / 3


def test_p_and_d_eri_by_centre_derivatives(oracle_lib):
    """Raw Gaussians obey d/dA_x e^{-a|r-A|^2} = 2a (x-A_x) e^{-a|r-A|^2}, so a
    p integral is a scaled centre derivative of an s integral, and d_xx / d_xy
    follow from p the same way.  With unit-normalised primitives:
      (p_x s|ss) = d/dA_x (s s|ss) / sqrt(a)
      (d_xx s|ss) = sqrt(a/3) * [d/dA_x (p_x s|ss) + 2 sqrt(a) (s s|ss)] / a ... (see below)."""
    import oracle
    rng = np.random.default_rng(5)
    ex = rng.uniform(0.3, 1.5, size=4)
    cen = rng.uniform(-1.0, 1.0, size=(4, 3))

    def eri(ls, A):
        c = cen.copy()
        c[0] = A
        return oracle.Basis(_prim_mol(ls, ex, c)).eri_shell(0, 1, 2, 3)

    a = ex[0]
    h = 1e-3
    ps = eri([1, 0, 0, 0], cen[0])[:, 0, 0, 0]
    for ax in range(3):
        def f(t, ax=ax):
            A = cen[0].copy()
            A[ax] += t
            return eri([0, 0, 0, 0], A)[0, 0, 0, 0]
        fd = _richardson(f, h) / np.sqrt(a)
        assert abs(ps[ax] - fd) < 2e-9 * max(1.0, abs(fd)), (ax, ps[ax], fd)

    # raw d_xx = (d/dA_x raw p_x + raw s) / (2a); raw d_xy = d/dA_y raw p_x / (2a)
    # norms: N_s = (2a/pi)^{3/4}, N_p = N_s 2 sqrt(a), N_dxx = N_s 4a / sqrt(3), N_dxy = N_s 4a
    ns = (2 * a / np.pi) ** 0.75
    np_ = ns * 2 * np.sqrt(a)
    ds = eri([2, 0, 0, 0], cen[0])[:, 0, 0, 0]
    ss = eri([0, 0, 0, 0], cen[0])[0, 0, 0, 0]

    def fpx(t, ax):
        A = cen[0].copy()
        A[ax] += t
        return eri([1, 0, 0, 0], A)[0, 0, 0, 0]

    raw_dxx = (_richardson(lambda t: fpx(t, 0), h) / np_ + ss / ns) / (2 * a)
    raw_dxy = (_richardson(lambda t: fpx(t, 1), h) / np_) / (2 * a)
    assert abs(ds[0] - ns * 4 * a / np.sqrt(3) * raw_dxx) < 2e-8 * abs(ds[0]) + 1e-10
    assert abs(ds[1] - ns * 4 * a * raw_dxy) < 2e-8 * abs(ds[1]) + 1e-10


def test_nuclear_attraction_p_by_centre_derivative(oracle_lib):
    import oracle
    ex = [0.9, 0.5]
    cen = np.array([[0.1, -0.2, 0.3], [0.7, 0.4, -0.5]])
    nuc = np.array([[-0.3, 0.6, 0.2]])

    def V(ls, A):
        c = cen.copy()
        c[0] = A
        shells = [W.Shell(0, ls[0], np.array([ex[0]]), np.array([1.0])),
                  W.Shell(1, ls[1], np.array([ex[1]]), np.array([1.0]))]
        allxyz = np.concatenate([c, nuc])
        m = W.Molecule(np.array([0, 0, 3], dtype=np.int32), allxyz, shells)
        return oracle.Basis(m).one_electron()[2]

    pv = V([1, 0], cen[0])[:3, 3]
    for ax in range(3):
        def f(t, ax=ax):
            A = cen[0].copy()
            A[ax] += t
            return V([0, 0], A)[0, 1]
        assert abs(pv[ax] - _richardson(f, 1e-3) / np.sqrt(ex[0])) < 1e-9


# ---- symmetry, Schwarz, enumeration, J/K ------------------------------------------------

@pytest.fixture(scope="module")
def dimer():
    import oracle
    m = W.dimer_config()
    return m, oracle.Basis(m)


def test_eri_8fold_symmetry_and_schwarz(dimer):
    _, B = dimer
    eri = B.eri_full()
    perms = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
             (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]
    for p in perms[1:]:
        assert np.abs(eri - eri.transpose(p)).max() <= 1e-15 * np.abs(eri).max() * 10
    n = eri.shape[0]
    diag = np.einsum("ijij->ij", eri)
    bound = np.sqrt(np.abs(diag)[:, :, None, None] * np.abs(diag)[None, None, :, :])
    assert (np.abs(eri) <= bound * (1 + 1e-12) + 1e-16).all()
    assert (diag >= -1e-15).all()
    assert n == 26


def test_unique_quartet_count(oracle_lib):
    import oracle
    for nsh in (1, 2, 5, 12, 40):
        shells = [W.Shell(i, 0, np.array([0.5 + 0.01 * i]), np.array([1.0])) for i in range(nsh)]
        cen = np.array([[0.3 * i, 0.0, 0.0] for i in range(nsh)])
        m = W.Molecule(np.zeros(nsh, dtype=np.int32), cen, shells)
        B = oracle.Basis(m)
        _, _, st = B.jk(np.eye(nsh), tau=0.0)
        P = nsh * (nsh + 1) // 2
        assert st[0] == P * (P + 1) // 2


def test_jk_8fold_equals_brute_force(dimer):
    m, B = dimer
    D = W.random_symmetric(m.nbf, 3)
    for tau in (0.0, 1e-10, 1e-4):
        J8, K8, _ = B.jk(D, tau)
        Jb, Kb = B.jk_brute(D, tau)
        assert np.abs(J8 - Jb).max() <= 1e-13 * max(1.0, np.abs(Jb).max())
        assert np.abs(K8 - Kb).max() <= 1e-13 * max(1.0, np.abs(Kb).max())
    # against the explicit N^4 tensor contraction (unscreened)
    eri = B.eri_full()
    J, K, _ = B.jk(D, 0.0)
    assert np.allclose(J, np.einsum("mnls,ls->mn", eri, D), atol=1e-12, rtol=0)
    assert np.allclose(K, np.einsum("mlns,ls->mn", eri, D), atol=1e-12, rtol=0)


def test_jk_block_equals_full(dimer):
    m, B = dimer
    D = W.random_symmetric(m.nbf, 4)
    J, K, _ = B.jk(D, 1e-10)
    bf = B.shell_bf
    for (a, b) in [(0, 0), (4, 1), (17, 9), (8, 3)]:
        Jb, Kb = B.jk_block(a, b, D, 1e-10)
        na, nb = Jb.shape
        assert np.abs(Jb - J[bf[a]:bf[a] + na, bf[b]:bf[b] + nb]).max() < 1e-13
        assert np.abs(Kb - K[bf[a]:bf[a] + na, bf[b]:bf[b] + nb]).max() < 1e-13


def test_jk_linearity_symmetry_positivity(dimer):
    m, B = dimer
    D1 = W.random_symmetric(m.nbf, 5)
    D2 = W.random_symmetric(m.nbf, 6)
    J1, K1, _ = B.jk(D1, 0.0)
    J2, K2, _ = B.jk(D2, 0.0)
    J3, K3, _ = B.jk(0.7 * D1 - 1.3 * D2, 0.0)
    assert np.allclose(J3, 0.7 * J1 - 1.3 * J2, atol=1e-12)
    assert np.allclose(K3, 0.7 * K1 - 1.3 * K2, atol=1e-12)
    assert np.abs(J1 - J1.T).max() < 1e-13 and np.abs(K1 - K1.T).max() < 1e-13
    Dp = W.random_orthonormal_density(m.nbf, 10, 8)
    J, K, _ = B.jk(Dp, 0.0)
    assert np.sum(Dp * J) >= np.sum(Dp * K) >= 0.0


# ---- SCF invariances --------------------------------------------------------------------

def _moved(m, R=None, t=None):
    import copy
    m2 = copy.deepcopy(m)
    xyz = m2.xyz.copy()
    if R is not None:
        xyz = xyz @ R.T
    if t is not None:
        xyz = xyz + t
    m2.xyz = xyz
    return m2


def test_scf_dimer_invariances(dimer):
    from oracle import scf
    m, B = dimer
    kw = dict(tau=0.0, e_tol=1e-11, d_tol=1e-9)
    r0 = scf.rhf(m, **kw)
    assert r0.converged
    S, _, _, _ = B.one_electron()
    assert abs(np.sum(r0.D * S) - m.nocc) < 1e-10
    rt = scf.rhf(_moved(m, t=np.array([0.7, -1.9, 3.3])), **kw)
    assert abs(rt.energy - r0.energy) < 1e-10
    R = W.random_rotation(np.random.default_rng(99))
    rr = scf.rhf(_moved(m, R=R), **kw)
    assert abs(rr.energy - r0.energy) < 1e-10


def test_sad_atomic_densities():
    from oracle import scf
    for z, basis in ((8, W.BASIS_SPD), (1, W.BASIS_SPD), (8, W.BASIS_SP)):
        shells = [W.Shell(0, l, np.array(e), np.array(c)) for (l, e, c) in basis[z]]
        D = scf.atomic_density(z, shells)
        import oracle
        mol = W.Molecule(np.array([z], dtype=np.int32), np.zeros((1, 3)), shells)
        S = oracle.Basis(mol).one_electron()[0]
        assert abs(np.sum(D * S) - z / 2.0) < 1e-10


def test_fractional_occupation_rule():
    from oracle import scf
    eps = np.array([-2.0, -1.0, -0.5, -0.5 + 1e-6, -0.5 - 1e-6, 0.3])
    occ = scf.fractional_occupation(eps, 4.0)
    assert np.allclose(occ, [1, 1, 2 / 3, 2 / 3, 2 / 3, 0])
    assert np.allclose(scf.fractional_occupation(np.array([-0.5, 0.1]), 0.5), [0.5, 0])


# ---- d shells on either side, Schwarz bounds ------------------------------------------

def _norm_comp(a, comp):
    """Unit-normalised Cartesian primitive factor (2a/pi)^{3/4} (4a)^{l/2} /
    sqrt((2lx-1)!!(2ly-1)!!(2lz-1)!!)."""
    def dfo(n):
        return float(np.prod(np.arange(2 * n - 1, 0, -2))) if n > 0 else 1.0
    l = sum(comp)
    return (2 * a / np.pi) ** 0.75 * (4 * a) ** (l / 2) / np.sqrt(dfo(comp[0]) * dfo(comp[1]) * dfo(comp[2]))


def _comps(l):
    return [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]


def _raise_by_derivative(l, comp_value, comp_value_at, a, h=1e-3):
    """Every raw component of angular momentum l from the raw components of
    l - 1 (and l - 2) on the same centre: for a raw Gaussian
    G_e = prod (x_i - A_i)^{e_i} exp(-a |r - A|^2),
      d/dA_i G_e = 2a G_{e + 1_i} - e_i G_{e - 1_i},
    so G_{e + 1_i} = (d/dA_i G_e + e_i G_{e - 1_i}) / (2a).
    comp_value(e) -> raw integral with the shell at its own centre;
    comp_value_at(e, i, t) -> the same with the centre moved by t along i.
    Returns {component: raw value}."""
    out = {}
    for e in _comps(l):
        i = next(k for k in range(3) if e[k] > 0)
        low = list(e)
        low[i] -= 1
        low = tuple(low)
        d = _richardson(lambda t: comp_value_at(low, i, t), h)
        extra = 0.0
        if low[i] > 0:
            lower2 = list(low)
            lower2[i] -= 1
            extra = low[i] * comp_value(tuple(lower2))
        out[e] = (d + extra) / (2 * a)
    return out


def test_eri_d_on_ket_by_centre_derivatives(oracle_lib):
    """(ss|ps) and (ss|ds) with the p/d shell on the ket side: centre
    derivatives of the lower-l integrals at centre C (shell index 2)."""
    import oracle
    rng = np.random.default_rng(17)
    ex = rng.uniform(0.3, 1.4, size=4)
    cen = rng.uniform(-1.0, 1.0, size=(4, 3))
    c_exp = ex[2]

    def raw(e, i=None, t=0.0):
        l = sum(e)
        c = cen.copy()
        if i is not None:
            c[2, i] += t
        blk = oracle.Basis(_prim_mol([0, 0, l, 0], ex, c)).eri_shell(0, 1, 2, 3)[0, 0, :, 0]
        k = _comps(l).index(e)
        return blk[k] / _norm_comp(c_exp, e)

    for l in (1, 2):
        got = oracle.Basis(_prim_mol([0, 0, l, 0], ex, cen)).eri_shell(0, 1, 2, 3)[0, 0, :, 0]
        ref = _raise_by_derivative(l, lambda e: raw(e), lambda e, i, t: raw(e, i, t), c_exp)
        for k, e in enumerate(_comps(l)):
            want = _norm_comp(c_exp, e) * ref[e]
            assert abs(got[k] - want) < 3e-8 * max(abs(want), 1e-3), (l, e, got[k], want)


@pytest.mark.parametrize("lket", [0, 1, 2])
def test_nuclear_attraction_d_by_centre_derivative(oracle_lib, lket):
    """d-shell nuclear attraction <d|V_C|X> (X = s, p, d) from centre
    derivatives of <p|V_C|X> and <s|V_C|X>."""
    import oracle
    ex = [0.85, 0.55]
    cen = np.array([[0.1, -0.2, 0.3], [0.7, 0.4, -0.5]])
    nuc = np.array([[-0.3, 0.6, 0.2]])
    nb = W.NCART[lket]

    def V(la, A):
        c = cen.copy()
        c[0] = A
        shells = [W.Shell(0, la, np.array([ex[0]]), np.array([1.0])),
                  W.Shell(1, lket, np.array([ex[1]]), np.array([1.0]))]
        m = W.Molecule(np.array([0, 0, 5], dtype=np.int32), np.concatenate([c, nuc]), shells)
        v = oracle.Basis(m).one_electron()[2]
        na = W.NCART[la]
        return v[:na, na:na + nb]

    for j in range(nb):
        def raw(e, i=None, t=0.0, j=j):
            A = cen[0].copy()
            if i is not None:
                A[i] += t
            l = sum(e)
            return V(l, A)[_comps(l).index(e), j] / _norm_comp(ex[0], e)

        got = V(2, cen[0])[:, j]
        ref = _raise_by_derivative(2, lambda e: raw(e), lambda e, i, t: raw(e, i, t), ex[0])
        for k, e in enumerate(_comps(2)):
            want = _norm_comp(ex[0], e) * ref[e]
            assert abs(got[k] - want) < 3e-8 * max(abs(want), 1e-3), (lket, j, e, got[k], want)


@pytest.fixture(scope="module")
def water_spd():
    """One water with the s/p/d basis (19 functions, d shell on oxygen)."""
    import oracle
    m = W.water_cluster(1, 5)
    return m, oracle.Basis(m)


def test_eri_8fold_symmetry_and_schwarz_spd(water_spd):
    """Every permutation symmetry and the Cauchy-Schwarz inequality with d
    shells on the bra and on the ket side."""
    _, B = water_spd
    eri = B.eri_full()
    assert eri.shape[0] == 19
    scale = np.abs(eri).max()
    for p in [(1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2), (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]:
        assert np.abs(eri - eri.transpose(p)).max() <= 1e-14 * scale, p
    diag = np.einsum("ijij->ij", eri)
    assert (diag >= -1e-15).all()
    bound = np.sqrt(np.abs(diag)[:, :, None, None] * np.abs(diag)[None, None, :, :])
    assert (np.abs(eri) <= bound * (1 + 1e-12) + 1e-16).all()


@pytest.mark.parametrize("which", ["dimer", "water_spd"])
def test_schwarz_bounds_equal_eri_diagonal(which, dimer, water_spd):
    """Q_ab = sqrt(max over mu in a, nu in b of (mu nu|mu nu)) read off the
    full ERI tensor (an independent route: every function quartet, no shell
    blocks)."""
    _, B = dimer if which == "dimer" else water_spd
    eri = B.eri_full()
    Q = B.schwarz()
    bf = list(B.shell_bf) + [B.nbf]
    diag = np.einsum("ijij->ij", eri)
    for a in range(B.nshell):
        for b in range(B.nshell):
            blk = diag[bf[a]:bf[a + 1], bf[b]:bf[b + 1]]
            assert abs(Q[a, b] - np.sqrt(blk.max())) <= 1e-14 * max(1.0, Q[a, b]), (a, b)
    assert np.abs(Q - Q.T).max() == 0.0


def test_jk_8fold_equals_brute_force_spd(water_spd):
    """The 8-fold loop with d shells: equal to the ordered brute force and to
    the N^4 tensor contraction."""
    m, B = water_spd
    D = W.random_symmetric(m.nbf, 31)
    J8, K8, _ = B.jk(D, 0.0)
    Jb, Kb = B.jk_brute(D, 0.0)
    assert np.abs(J8 - Jb).max() <= 1e-13 * np.abs(Jb).max()
    assert np.abs(K8 - Kb).max() <= 1e-13 * np.abs(Kb).max()
    eri = B.eri_full()
    assert np.allclose(J8, np.einsum("mnls,ls->mn", eri, D), atol=1e-12, rtol=0)
    assert np.allclose(K8, np.einsum("mlns,ls->mn", eri, D), atol=1e-12, rtol=0)


# ---- SP shells and the graphene workload -----------------------------------------------

def test_sp_shell_is_an_s_and_a_p_shell(oracle_lib):
    """An SP (L) shell is by definition an s and a p shell sharing its
    exponents: integrals over a molecule with SP shells equal those with the
    two shells written out (s coefficients, then p coefficients)."""
    import oracle
    base = W.graphene_bilayer(1)   # two carbons, one per layer
    ex = []
    for sh in base.shells:
        if sh.l == W.SP:
            ex.append(W.Shell(sh.atom, 0, sh.exps, sh.coefs))
            ex.append(W.Shell(sh.atom, 1, sh.exps, sh.coefs_p))
        else:
            ex.append(sh)
    written = W.Molecule(base.Z.copy(), base.xyz.copy(), ex)
    Bsp, Bex = oracle.Basis(base), oracle.Basis(written)
    assert Bsp.nbf == Bex.nbf == 30 and Bsp.nshell == Bex.nshell == 12
    for a, b in zip(Bsp.one_electron(), Bex.one_electron()):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    D = W.random_symmetric(30, 7, 0.3)
    J1, K1, s1 = Bsp.jk(D, 0.0)
    J2, K2, s2 = Bex.jk(D, 0.0)
    assert s1 == s2   # the same quartets; sums agree up to the threads' summation order
    assert np.abs(J1 - J2).max() <= 1e-14 * np.abs(J1).max() and np.abs(K1 - K2).max() <= 1e-14 * np.abs(K1).max()
    # the SP shell's s and p parts use their own coefficients
    S = Bsp.one_electron()[0]
    assert np.allclose(np.diag(S), 1.0, atol=1e-13)


def test_graphene_sizes_match_the_papers_table():
    """Atoms, shells and basis functions of the five bilayers equal the
    paper's table of chemical systems (appendix A, Table 4: 44/176/660,
    120/480/1,800, 220/880/3,300, 356/1,424/5,340, 2,016/8,064/30,240)."""
    table = {"0.5nm": (44, 176, 660), "1nm": (120, 480, 1800), "1.5nm": (220, 880, 3300),
             "2nm": (356, 1424, 5340), "5nm": (2016, 8064, 30240)}
    for name, n in W.GRAPHENE_SIZES.items():
        m = W.graphene_bilayer(n)
        assert (m.natom, m.nshell, m.nbf) == table[name], name
        xyz = m.xyz / W.ANGSTROM_TO_BOHR
        lay = xyz[:, 2] < 1.0
        assert lay.sum() == n
        d = np.sqrt(((xyz[lay][:, None] - xyz[lay][None]) ** 2).sum(-1)) + 9 * np.eye(n)
        assert abs(d.min() - W.CC_BOND) < 1e-12          # honeycomb bond length within a layer
        assert abs(xyz[~lay, 2].min() - W.INTERLAYER) < 1e-12
