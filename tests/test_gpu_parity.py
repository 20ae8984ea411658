"""GPU parity: the HIP library (through its C ABI) against the CPU oracle
on the same seeded inputs."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _hfx():
    from paper_1708_00033_amd import hfx
    return hfx


@pytest.fixture(scope="module")
def dimer():
    import oracle
    m = W.dimer_config()
    B = oracle.Basis(m)
    return m, B


@pytest.fixture(scope="module")
def four_waters():
    """Four waters with the d shell: every one of the 21 quartet classes."""
    import oracle
    m = W.water_cluster(4, 41)
    return m, oracle.Basis(m)


def _fock_ref(B, D, tau=1e-10):
    S, T, V, _ = B.one_electron()
    J, K, _ = B.jk(D, tau)
    return T + V + 2 * J - K, J, K


def test_one_electron_and_schwarz(four_waters):
    m, B = four_waters
    ctx = _hfx().Context().load(m)
    S, H, enuc = ctx.core()
    So, To, Vo, eo = B.one_electron()
    assert np.abs(S - So).max() < 1e-12
    assert np.abs(H - (To + Vo)).max() < 1e-10
    assert abs(enuc - eo) < 1e-10
    Q = ctx.schwarz()
    Qo = B.schwarz()
    assert np.allclose(Q, Qo, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("digest", [0, 1])
def test_fock_parity_dimer(dimer, digest):
    m, B = dimer
    ctx = _hfx().Context(digest=digest).load(m)
    for seed in (1, 2):
        D = W.random_symmetric(m.nbf, seed, 0.2)
        F, st = ctx.build_fock(D)
        ref, _, _ = _fock_ref(B, D)
        assert np.abs(F - ref).max() < 1e-10, np.abs(F - ref).max()
        assert st.quartets_fp64 == 14706


@pytest.mark.parametrize("digest", [0, 1])
@pytest.mark.parametrize("task", [256, 2048])
def test_fock_parity_all_classes(four_waters, digest, task):
    m, B = four_waters
    ctx = _hfx().Context(digest=digest, task_quartets=task).load(m)
    D = W.random_symmetric(m.nbf, 7, 0.2)
    F, st = ctx.build_fock(D)
    ref, J, K = _fock_ref(B, D)
    err = np.abs(F - ref).max()
    assert err < 1e-10 * max(1.0, np.abs(ref).max()), err
    _, _, ost = B.jk(D, 1e-10)
    assert st.quartets_fp64 == ost[0]
    assert st.integrals == ost[1]
    counts = ctx.class_counts()
    assert (counts[:, 0] > 0).all(), "every class must be exercised"


def test_j_and_k_separately(four_waters):
    import torch
    m, B = four_waters
    ctx = _hfx().Context().load(m)
    D = W.random_symmetric(m.nbf, 9, 0.2)
    dD = torch.tensor(D, device="cuda")
    dG = torch.empty_like(dD)
    s = torch.cuda.current_stream().cuda_stream
    _, J, K = _fock_ref(B, D)
    ctx.build_2e_dev(dD.data_ptr(), 1.0, 0.0, dG.data_ptr(), s)
    torch.cuda.synchronize()
    assert np.abs(dG.cpu().numpy() - J).max() < 1e-10
    ctx.build_2e_dev(dD.data_ptr(), 0.0, -1.0, dG.data_ptr(), s)
    torch.cuda.synchronize()
    assert np.abs(dG.cpu().numpy() - K).max() < 1e-10


def test_scf_energy_dimer(dimer):
    from oracle import scf
    m, _ = dimer
    ref = scf.rhf(m, tau=1e-10, e_tol=1e-11, d_tol=1e-9)
    ctx = _hfx().Context().load(m)
    r = ctx.scf(e_tol=1e-11, d_rms_tol=1e-9)
    assert r["converged"]
    assert abs(r["energy"] - ref.energy) < 1e-9, (r["energy"], ref.energy)
    assert np.abs(r["D"] - ref.D).max() < 1e-6


def test_mixed_precision_dimer(dimer):
    m, B = dimer
    ctx64 = _hfx().Context().load(m)
    r64 = ctx64.scf(e_tol=1e-10, d_rms_tol=1e-8)
    ctx = _hfx().Context(precision=1).load(m)
    F, st = ctx.build_fock(r64["D"])
    F64, _ = ctx64.build_fock(r64["D"])
    assert st.quartets_fp32 > 0
    assert np.abs(F - F64).max() < 1e-5
    r = ctx.scf(e_tol=1e-10, d_rms_tol=1e-8)
    assert abs(r["energy"] - r64["energy"]) < 1e-6


def test_invalid_inputs():
    hfx = _hfx()
    ctx = hfx.Context()
    m = W.dimer_config()
    bad = W.Molecule(m.Z.copy(), m.xyz.copy(), [W.Shell(0, 3, np.array([1.0]), np.array([1.0]))])
    with pytest.raises(hfx.HfxError) as e:
        ctx.load(bad)
    assert e.value.status == hfx.HFX_ERR_INVALID_ARG
    bad = W.Molecule(m.Z.copy(), m.xyz.copy(), [W.Shell(0, 0, np.array([-1.0]), np.array([1.0]))])
    with pytest.raises(hfx.HfxError):
        ctx.load(bad)
    xyz = m.xyz.copy()
    xyz[0, 0] = np.nan
    with pytest.raises(hfx.HfxError):
        ctx.load(W.Molecule(m.Z.copy(), xyz, m.shells))
    ctx.load(m)
    D = np.zeros((m.nbf, m.nbf))
    D[0, 0] = np.nan
    with pytest.raises(hfx.HfxError) as e:
        ctx.build_fock(D)
    assert e.value.status == hfx.HFX_ERR_NUMERICAL
