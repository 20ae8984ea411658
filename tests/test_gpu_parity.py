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


@pytest.mark.parametrize("digest", [0, 1, 3])
def test_fock_parity_dimer(dimer, digest):
    m, B = dimer
    ctx = _hfx().Context(digest=digest).load(m)
    for seed in (1, 2):
        D = W.random_symmetric(m.nbf, seed, 0.2)
        F, st = ctx.build_fock(D)
        ref, _, _ = _fock_ref(B, D)
        assert np.abs(F - ref).max() < 1e-10, np.abs(F - ref).max()
        assert st.quartets_fp64 == 14706


@pytest.mark.parametrize("digest", [0, 1, 3])
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
    assert st.quartets_fp32 + st.quartets_fp64 == 14706
    assert np.abs(F - F64).max() < 1e-5
    r = ctx.scf(e_tol=1e-10, d_rms_tol=1e-8)
    assert abs(r["energy"] - r64["energy"]) < 1e-6


@pytest.mark.parametrize("persistent,digest", [(0, -1), (1, -1), (0, 1), (1, 1), (2, -1), (1, 0), (2, 0)])
def test_mixed_precision_16_waters(persistent, digest):
    """A mixed build evaluates each task's kets before its split in FP64 and
    the rest in FP32, in one launch; a 16-water cluster puts a large share in
    FP32.  Every launch form and both digestions agree with FP64 within
    tolerance."""
    m = W.water_cluster(16, 77)
    D = W.random_orthonormal_density(m.nbf, m.nocc, 5)
    F64, s64 = _hfx().Context().load(m).build_fock(D)
    ctx = _hfx().Context(precision=1).load(m)
    ctx.set_class_tuning(-1, 2048, 1, persistent, digest)
    Fmx, smx = ctx.build_fock(D)
    assert smx.quartets_fp32 + smx.quartets_fp64 == s64.quartets_fp64
    assert smx.quartets_fp32 > 0.2 * s64.quartets_fp64
    assert np.abs(Fmx - F64).max() < 1e-6
    assert abs(np.sum(D * (Fmx - F64))) < 1e-6


def test_precision_autotuner_keeps_tolerance():
    """Per-class FP32 choice (autotuned or forced off) changes only which
    eligible quartets run in FP32: FP64-only equals the FP64 build."""
    import torch
    from paper_1708_00033_amd import autotune
    m = W.water_cluster(16, 78)
    D = W.random_orthonormal_density(m.nbf, m.nocc, 6)
    F64, s64 = _hfx().Context().load(m).build_fock(D)
    ctx = _hfx().Context(precision=1).load(m)
    dD = torch.tensor(D, device="cuda")
    dF = torch.empty_like(dD)
    s = torch.cuda.current_stream().cuda_stream
    table = autotune.autotune_precision(ctx, dD.data_ptr(), dF.data_ptr(), s, reps=1)
    assert set(table) == set(_hfx().CLASS_NAMES)
    Fmx, smx = ctx.build_fock(D)
    assert smx.quartets_fp32 + smx.quartets_fp64 == s64.quartets_fp64
    assert np.abs(Fmx - F64).max() < 1e-6
    ctx.set_class_precision(-1, 0)
    Fo, so = ctx.build_fock(D)
    assert so.quartets_fp32 == 0
    assert np.abs(Fo - F64).max() <= 1e-13 * np.abs(F64).max()


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


def test_determinism_and_partition_invariance(four_waters):
    import torch
    m, _ = four_waters
    ctx = _hfx().Context().load(m)
    D = W.random_symmetric(m.nbf, 11, 0.2)
    dD = torch.tensor(D, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    G1, G2 = torch.empty_like(dD), torch.empty_like(dD)
    ctx.build_2e_dev(dD.data_ptr(), 2.0, 1.0, G1.data_ptr(), s)
    ctx.build_2e_dev(dD.data_ptr(), 2.0, 1.0, G2.data_ptr(), s)
    torch.cuda.synchronize()
    scale = G1.abs().max().item()
    assert (G1 - G2).abs().max().item() <= 1e-13 * scale
    for nshards in (2, 3, 7):
        tot = torch.zeros_like(dD)
        part = torch.empty_like(dD)
        for g in range(nshards):
            ctx.build_2e_shard_dev(dD.data_ptr(), 2.0, 1.0, g, nshards, part.data_ptr(), s)
            tot += part
        torch.cuda.synchronize()
        assert (tot - G1).abs().max().item() <= 1e-13 * scale


def test_h2_textbook_on_gpu():
    m = W.h2(1.4)
    ctx = _hfx().Context().load(m)
    r = ctx.scf(guess=_hfx().HFX_GUESS_CORE, e_tol=1e-12, d_rms_tol=1e-10)
    assert abs(r["energy"] - (-1.1167143250625697)) < 1e-10
    counts = ctx.class_counts()
    assert counts[0, 0] == 6 and counts[1:, 0].sum() == 0   # (ss|ss) only: P(P+1)/2 with P = 3


def test_single_water_and_tiny_tasks():
    import oracle
    m = W.water_cluster(1, 5)
    B = oracle.Basis(m)
    ctx = _hfx().Context(task_quartets=256).load(m)
    D = W.random_symmetric(m.nbf, 12, 0.3)
    F, st = ctx.build_fock(D)
    ref, _, _ = _fock_ref(B, D)
    assert np.abs(F - ref).max() < 1e-10
    r = ctx.scf(e_tol=1e-10, d_rms_tol=1e-8)
    from oracle import scf
    ro = scf.rhf(m, tau=1e-10, e_tol=1e-10, d_tol=1e-8)
    assert abs(r["energy"] - ro.energy) < 1e-8


def test_screening_threshold_edge(dimer):
    """A huge tau keeps only the strongest quartets; zero tau keeps all."""
    m, B = dimer
    for tau in (0.0, 1e-3):
        ctx = _hfx().Context(schwarz_tau=tau).load(m)
        D = W.random_symmetric(m.nbf, 13, 0.2)
        F, st = ctx.build_fock(D)
        S, T, V, _ = B.one_electron()
        J, K, ost = B.jk(D, tau)
        assert st.quartets_fp64 == ost[0]
        assert np.abs(F - (T + V + 2 * J - K)).max() < 1e-10


def test_cluster64_sampled_blocks():
    """Full-size 64-water build with the library's default launch forms
    (static workgroup tasks; the benchmark's autotuned persistent forms are
    covered against the stored oracle golden in test_gpu_fp32_full), checked
    on four shell blocks of J and K that the oracle computes one by one."""
    import torch
    import oracle
    m = W.cluster64_config()
    ctx = _hfx().Context().load(m)
    D = W.random_orthonormal_density(m.nbf, m.nocc, 21)
    dD = torch.tensor(D, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    J, K = torch.empty_like(dD), torch.empty_like(dD)
    ctx.build_2e_dev(dD.data_ptr(), 1.0, 0.0, J.data_ptr(), s)
    ctx.build_2e_dev(dD.data_ptr(), 0.0, -1.0, K.data_ptr(), s)
    torch.cuda.synchronize()
    J, K = J.cpu().numpy(), K.cpu().numpy()
    B = oracle.Basis(m)
    bf = B.shell_bf
    ls = B.shell_l
    picks = [0, 3, 5, 211, 639]   # s, p, d shells across the cluster
    for a, b in [(picks[0], picks[1]), (picks[2], picks[2]), (picks[3], picks[4]), (picks[1], picks[4])]:
        Jb, Kb = B.jk_block(a, b, D, 1e-10)
        na, nb = Jb.shape
        assert np.abs(J[bf[a]:bf[a] + na, bf[b]:bf[b] + nb] - Jb).max() < 1e-10, (a, b)
        assert np.abs(K[bf[a]:bf[a] + na, bf[b]:bf[b] + nb] - Kb).max() < 1e-10, (a, b)
    assert ls[5] == 2 and ls[3] == 1


def test_windowed_lds_digestion_112_waters():
    """Above 2048 basis functions the LDS bra rows cover two column windows
    per task (kets grouped by the windows of their shells): the whole J and K
    equal the global-atomic digestion's, sampled blocks equal the oracle's,
    and a mixed build (per-task FP32 split) stays within tolerance."""
    import torch
    import oracle
    m = W.water_cluster(112, 5)
    assert m.nbf > 2048
    D = W.random_orthonormal_density(m.nbf, m.nocc, 23)
    dD = torch.tensor(D, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    out = {}
    for digest in (0, 1, 3):
        ctx = _hfx().Context(digest=digest).load(m)
        J, K = torch.empty_like(dD), torch.empty_like(dD)
        ctx.build_2e_dev(dD.data_ptr(), 1.0, 0.0, J.data_ptr(), s)
        ctx.build_2e_dev(dD.data_ptr(), 0.0, -1.0, K.data_ptr(), s)
        torch.cuda.synchronize()
        out[digest] = (J.cpu().numpy(), K.cpu().numpy())
        if digest == 0:
            assert {p["mode"] for p in ctx.plans()} >= {0}
        if digest == 3:   # with column windows the rows of D are not staged
            assert {p["mode"] for p in ctx.plans()} <= {0, 1}
    (J0, K0), (J1, K1), (J3, K3) = out[0], out[1], out[3]
    assert np.abs(J0 - J1).max() <= 1e-12 * np.abs(J1).max()
    assert np.abs(K0 - K1).max() <= 1e-12 * np.abs(K1).max()
    assert np.abs(J3 - J1).max() <= 1e-12 * np.abs(J1).max()
    assert np.abs(K3 - K1).max() <= 1e-12 * np.abs(K1).max()
    B = oracle.Basis(m)
    bf = B.shell_bf
    for a, b in [(0, 3), (5, 5), (700, 1115), (1000, 13)]:
        Jb, Kb = B.jk_block(a, b, D, 1e-10)
        na, nb = Jb.shape
        assert np.abs(J0[bf[a]:bf[a] + na, bf[b]:bf[b] + nb] - Jb).max() < 1e-10, (a, b)
        assert np.abs(K0[bf[a]:bf[a] + na, bf[b]:bf[b] + nb] - Kb).max() < 1e-10, (a, b)
    ctx = _hfx().Context(precision=1).load(m)
    G = torch.empty_like(dD)
    st = ctx.build_2e_dev(dD.data_ptr(), 2.0, 1.0, G.data_ptr(), s, stats=True)
    torch.cuda.synchronize()
    assert st.quartets_fp32 > 0
    assert np.abs(G.cpu().numpy() - (2 * J0 - K0)).max() < 1e-6


def test_launch_chunks_cover_every_task():
    """256-quartet tasks on the 64-water cluster give (ss|ss) more than 2^20
    workgroups, so its static launches are chunked below the 2^32 work-item
    grid limit: every planned quartet is evaluated and F is unchanged."""
    import torch
    m = W.cluster64_config()
    ctx = _hfx().Context().load(m)
    D = torch.tensor(W.random_orthonormal_density(m.nbf, m.nocc, 3), device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    ref = torch.empty_like(D)
    st0 = ctx.build_fock_dev(D.data_ptr(), ref.data_ptr(), s, stats=True)
    ctx.set_class_tuning(-1, 256, 0)
    assert max(p["tasks"] for p in ctx.plans()) > (1 << 20)
    out = torch.empty_like(D)
    st1 = ctx.build_fock_dev(D.data_ptr(), out.data_ptr(), s, stats=True)
    planned = int(ctx.class_counts()[:, 0].sum())
    assert st0.quartets_fp64 == planned and st1.quartets_fp64 == planned
    assert (out - ref).abs().max().item() <= 1e-13 * ref.abs().max().item()


def test_scheduling_knobs_do_not_change_results():
    """Task size, XCD striping and the launch form move work between workgroups (or waves) only."""
    import torch
    m = W.water_cluster(16, 77)
    ctx = _hfx().Context().load(m)
    D = torch.tensor(W.random_orthonormal_density(m.nbf, m.nocc, 5), device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    ref = torch.empty_like(D)
    ctx.set_class_tuning(-1, 256, 0)
    ctx.build_2e_dev(D.data_ptr(), 2.0, 1.0, ref.data_ptr(), s)
    out = torch.empty_like(D)
    for tq, st, pe, dg in [(8192, 1, 0, -1), (1024, 1, 0, -1), (32768, 0, 0, -1), (2048, 1, 1, -1),
                           (256, 0, 1, -1), (32768, 1, 1, -1), (8192, 0, 0, 1), (2048, 1, 1, 1),
                           (2048, 1, 2, -1), (32768, 0, 2, -1), (8192, 1, 2, 1),
                           (32768, 0, 3, -1), (2048, 1, 3, -1), (256, 0, 3, -1), (8192, 1, 3, 1),
                           (8192, 1, 0, 2), (2048, 1, 1, 2), (32768, 0, 2, 2), (2048, 0, 3, 2)]:
        ctx.set_class_tuning(-1, tq, st, pe, dg)
        ctx.build_2e_dev(D.data_ptr(), 2.0, 1.0, out.data_ptr(), s)
        torch.cuda.synchronize()
        assert (out - ref).abs().max().item() <= 1e-13 * ref.abs().max().item(), (tq, st, pe, dg)
    from paper_1708_00033_amd import autotune
    F = torch.empty_like(D)
    table = autotune.autotune(ctx, D.data_ptr(), F.data_ptr(), s, candidates=((512, 0), (4096, 1, 1), (2048, 0, 0, 1)),
                              reps=1)
    assert set(table) == set(_hfx().CLASS_NAMES)
    ctx.build_2e_dev(D.data_ptr(), 2.0, 1.0, out.data_ptr(), s)
    torch.cuda.synchronize()
    assert (out - ref).abs().max().item() <= 1e-13 * ref.abs().max().item()



def test_launch_streams_do_not_change_results():
    """Class launches dealt over 1..4 streams (eager, multi-density and graph-replayed builds) give the
    one-stream result up to the order of sums; the stream count is range-checked."""
    import torch
    hfx = _hfx()
    m = W.water_cluster(16, 78)
    ctx = hfx.Context().load(m)
    D = torch.tensor(W.random_orthonormal_density(m.nbf, m.nocc, 6), device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    for bad in (0, 5):
        with pytest.raises(RuntimeError):
            ctx.set_streams(bad)
    out = torch.empty_like(D)
    for prec in (hfx.HFX_PREC_FP64, hfx.HFX_PREC_MIXED):
        ctx.configure(precision=prec)
        ctx.set_streams(1)
        ref = torch.empty_like(D)
        ctx.build_fock_dev(D.data_ptr(), ref.data_ptr(), s)
        torch.cuda.synchronize()
        for ns in (2, 3, 4):
            ctx.set_streams(ns)
            st = ctx.build_fock_dev(D.data_ptr(), out.data_ptr(), s, stats=True)
            assert st.quartets_fp64 + st.quartets_fp32 == int(ctx.class_counts()[:, 0].sum())
            assert (out - ref).abs().max().item() <= 1e-13 * ref.abs().max().item(), (prec, ns)
    ctx.configure(precision=hfx.HFX_PREC_FP64)
    ctx.set_streams(1)
    ref = torch.empty_like(D)
    ctx.build_fock_dev(D.data_ptr(), ref.data_ptr(), s)
    DD = torch.stack([D, D.flip(0).flip(1)]).contiguous()
    J1, K1 = torch.empty_like(DD), torch.empty_like(DD)
    ctx.build_jk_multi_dev(2, DD.data_ptr(), J1.data_ptr(), K1.data_ptr(), s)
    ctx.set_streams(3)
    J3, K3 = torch.empty_like(DD), torch.empty_like(DD)
    ctx.build_jk_multi_dev(2, DD.data_ptr(), J3.data_ptr(), K3.data_ptr(), s)
    torch.cuda.synchronize()
    assert (J3 - J1).abs().max().item() <= 1e-13 * J1.abs().max().item()
    assert (K3 - K1).abs().max().item() <= 1e-13 * K1.abs().max().item()
    # captured with three streams: the side streams fork from and join into the capturing stream
    cs = torch.cuda.Stream()
    G = torch.zeros_like(D)
    ctx.graph_capture(D.data_ptr(), G.data_ptr(), cs.cuda_stream)
    for r in range(3):
        G.zero_()
        ctx.build_fock_dev(D.data_ptr(), out.data_ptr(), s)   # eager work between the replays
        torch.cuda.synchronize()
        ctx.graph_launch(cs.cuda_stream)
        torch.cuda.synchronize()
        assert (G - ref).abs().max().item() <= 1e-13 * ref.abs().max().item(), r
        assert (out - ref).abs().max().item() <= 1e-13 * ref.abs().max().item(), r

@pytest.mark.parametrize("digest", [0, 1])
def test_register_tiled_form_all_classes(four_waters, digest):
    """Launch form 3 (ket primitives in registers, blocks of two bras with
    per-lane screening) on every class that has it: F, the quartet count and
    the per-class counts equal the oracle's; classes without it fall back."""
    m, B = four_waters
    ctx = _hfx().Context(digest=digest).load(m)
    ctx.set_class_tuning(-1, 512, 1, 3, -1)
    plans = ctx.plans()
    assert any(p["persistent"] == 3 and p["bras_per_task"] == 2 for p in plans)
    D = W.random_symmetric(m.nbf, 71, 0.2)
    F, st = ctx.build_fock(D)
    ref, _, _ = _fock_ref(B, D)
    assert np.abs(F - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())
    _, _, ost = B.jk(D, 1e-10)
    assert st.quartets_fp64 == ost[0] and st.quartets_fp32 == 0
    # mixed: the register-tiled classes run FP64, the rest keep their split
    ctx.configure(precision=_hfx().HFX_PREC_MIXED)
    Fm, stm = ctx.build_fock(D)
    assert stm.quartets_fp64 + stm.quartets_fp32 == ost[0]
    assert np.abs(Fm - ref).max() < 1e-6


def test_register_tiled_form_batch_windows_and_shards():
    """Blocks of bras never cross molecules of a batch; with column windows
    (above 2048 basis functions) and with shards (bras of one block in
    different shards) the results equal the default form's."""
    import torch
    s = torch.cuda.current_stream().cuda_stream
    mols = [W.water_cluster(3, 81), W.water_cluster(1, 82), W.water_cluster(6, 83), W.water_cluster(2, 84)]
    ctx = _hfx().Context().load_batch(mols)
    nbf, nocc, off, tot = ctx.layout
    D = torch.tensor(np.concatenate([W.random_orthonormal_density(int(n), int(o), 40 + i).ravel()
                                     for i, (n, o) in enumerate(zip(nbf, nocc))]), device="cuda")
    ref, out = torch.empty_like(D), torch.empty_like(D)
    st0 = ctx.build_2e_dev(D.data_ptr(), 2.0, 1.0, ref.data_ptr(), s, stats=True)
    ctx.set_class_tuning(-1, 1024, 1, 3, -1)
    st1 = ctx.build_2e_dev(D.data_ptr(), 2.0, 1.0, out.data_ptr(), s, stats=True)
    torch.cuda.synchronize()
    assert st1.quartets_fp64 == st0.quartets_fp64
    assert (out - ref).abs().max().item() <= 1e-13 * ref.abs().max().item()
    for nshards in (2, 3):
        tot_ = torch.zeros_like(D)
        part = torch.empty_like(D)
        for g in range(nshards):
            ctx.build_2e_shard_dev(D.data_ptr(), 2.0, 1.0, g, nshards, part.data_ptr(), s)
            tot_ += part
        torch.cuda.synchronize()
        assert (tot_ - ref).abs().max().item() <= 1e-13 * ref.abs().max().item()
    m = W.water_cluster(112, 5)
    Dw = torch.tensor(W.random_orthonormal_density(m.nbf, m.nocc, 23), device="cuda")
    cw = _hfx().Context().load(m)
    rw, ow = torch.empty_like(Dw), torch.empty_like(Dw)
    cw.build_2e_dev(Dw.data_ptr(), 2.0, 1.0, rw.data_ptr(), s)
    cw.set_class_tuning(-1, 8192, 1, 3, -1)
    assert any(p["persistent"] == 3 for p in cw.plans())
    cw.build_2e_dev(Dw.data_ptr(), 2.0, 1.0, ow.data_ptr(), s)
    torch.cuda.synchronize()
    assert (ow - rw).abs().max().item() <= 1e-13 * rw.abs().max().item()


@pytest.mark.parametrize("persistent", [0, 1, 2])
def test_private_digestion_all_classes(four_waters, persistent):
    """Per-XCD private copies of the Fock matrix (algorithm 2's private Fock
    matrices, one per XCD) reduced after the class launches: F equals the
    oracle's for every class and launch form, and J, K separately."""
    import torch
    m, B = four_waters
    hfx = _hfx()
    ctx = hfx.Context(digest=hfx.HFX_DIGEST_PRIVATE).load(m)
    ctx.set_class_tuning(-1, 1024, 1, persistent, -1)
    assert {p["mode"] for p in ctx.plans()} == {2}
    D = W.random_symmetric(m.nbf, 73, 0.2)
    F, st = ctx.build_fock(D)
    ref, J, K = _fock_ref(B, D)
    assert np.abs(F - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())
    dD = torch.tensor(D, device="cuda")
    G = torch.empty_like(dD)
    s = torch.cuda.current_stream().cuda_stream
    ctx.build_2e_dev(dD.data_ptr(), 0.0, -1.0, G.data_ptr(), s)
    torch.cuda.synchronize()
    assert np.abs(G.cpu().numpy() - K).max() < 1e-10


def test_private_digestion_batch_and_mixed_with_other_digestions():
    """Per class a different digestion (LDS, shared global, private) in one
    build of a batch, FP64 and mixed: equal to the all-LDS build."""
    import torch
    hfx = _hfx()
    s = torch.cuda.current_stream().cuda_stream
    mols = [W.water_cluster(5, 85), W.water_cluster(2, 86)]
    ctx = hfx.Context().load_batch(mols)
    nbf, nocc, off, tot = ctx.layout
    D = torch.tensor(np.concatenate([W.random_orthonormal_density(int(n), int(o), 50 + i).ravel()
                                     for i, (n, o) in enumerate(zip(nbf, nocc))]), device="cuda")
    ref, out = torch.empty_like(D), torch.empty_like(D)
    ctx.build_2e_dev(D.data_ptr(), 2.0, 1.0, ref.data_ptr(), s)
    for k in range(21):
        ctx.set_class_tuning(k, 2048, 1, k % 3, [0, 1, 2][(k // 3) % 3])
    assert {p["mode"] for p in ctx.plans()} == {0, 1, 2}
    ctx.build_2e_dev(D.data_ptr(), 2.0, 1.0, out.data_ptr(), s)
    torch.cuda.synchronize()
    assert (out - ref).abs().max().item() <= 1e-13 * ref.abs().max().item()
    ctx.configure(precision=hfx.HFX_PREC_MIXED)
    st = ctx.build_2e_dev(D.data_ptr(), 2.0, 1.0, out.data_ptr(), s, stats=True)
    torch.cuda.synchronize()
    assert st.quartets_fp32 > 0
    assert (out - ref).abs().max().item() < 1e-6


def test_multi_density_jk_against_oracle(four_waters):
    """Three densities in one pass over the integrals: J(D_d) and K(D_d) of
    each equal the oracle's, the quartets are counted once, and an
    unrestricted alpha/beta Fock pair formed from them equals the one formed
    from single-density builds."""
    import torch
    m, B = four_waters
    hfx = _hfx()
    n = m.nbf
    Ds = [W.random_symmetric(n, 90 + d, 0.2) for d in range(3)]
    dD = torch.tensor(np.stack(Ds), device="cuda")
    dJ, dK = torch.empty_like(dD), torch.empty_like(dD)
    s = torch.cuda.current_stream().cuda_stream
    for tuning in [None, (512, 1, 3, -1), (1024, 1, 1, 2)]:
        ctx = hfx.Context().load(m)
        if tuning:
            ctx.set_class_tuning(-1, *tuning)
        st = ctx.build_jk_multi_dev(3, dD.data_ptr(), dJ.data_ptr(), dK.data_ptr(), s, stats=True)
        torch.cuda.synchronize()
        _, _, ost = B.jk(Ds[0], 1e-10)
        assert st.quartets_fp64 == ost[0]
        J, K = dJ.cpu().numpy(), dK.cpu().numpy()
        for d in range(3):
            Jo, Ko, _ = B.jk(Ds[d], 1e-10)
            assert np.abs(J[d] - Jo).max() < 1e-10, (tuning, d)
            assert np.abs(K[d] - Ko).max() < 1e-10, (tuning, d)
    # unrestricted pair from one pass vs from single-density builds
    Fa = J[0] + J[1] - K[0]
    G = torch.empty((n, n), dtype=torch.float64, device="cuda")
    ctx.build_2e_dev(dD[0].data_ptr(), 1.0, 1.0, G.data_ptr(), s)   # J_a - K_a
    Jb = torch.empty_like(G)
    ctx.build_2e_dev(dD[1].data_ptr(), 1.0, 0.0, Jb.data_ptr(), s)
    torch.cuda.synchronize()
    assert np.abs(Fa - (G + Jb).cpu().numpy()).max() < 1e-12 * np.abs(Fa).max()
    # only K requested
    dK2 = torch.empty_like(dD)
    ctx.build_jk_multi_dev(3, dD.data_ptr(), 0, dK2.data_ptr(), s)
    torch.cuda.synchronize()
    assert (dK2 - dK).abs().max().item() < 1e-12


def test_multi_density_batch_and_limits():
    """A batch (ragged layout per density) and argument checks."""
    import torch
    hfx = _hfx()
    import oracle
    mols = [W.water_cluster(2, 95), W.water_cluster(1, 96)]
    ctx = hfx.Context().load_batch(mols)
    nbf, nocc, off, tot = ctx.layout
    Ds = [np.concatenate([W.random_symmetric(int(nb), 100 + 10 * d + i, 0.2).ravel() for i, nb in enumerate(nbf)])
          for d in range(2)]
    dD = torch.tensor(np.stack(Ds), device="cuda")
    dJ, dK = torch.empty_like(dD), torch.empty_like(dD)
    s = torch.cuda.current_stream().cuda_stream
    ctx.build_jk_multi_dev(2, dD.data_ptr(), dJ.data_ptr(), dK.data_ptr(), s)
    torch.cuda.synchronize()
    J, K = dJ.cpu().numpy(), dK.cpu().numpy()
    for i, mol in enumerate(mols):
        Bm = oracle.Basis(mol)
        nb = int(nbf[i])
        sl = slice(int(off[i]), int(off[i]) + nb * nb)
        for d in range(2):
            Jo, Ko, _ = Bm.jk(Ds[d][sl].reshape(nb, nb), 1e-10)
            assert np.abs(J[d][sl].reshape(nb, nb) - Jo).max() < 1e-10
            assert np.abs(K[d][sl].reshape(nb, nb) - Ko).max() < 1e-10
    for bad in (0, 65):
        with pytest.raises(hfx.HfxError):
            ctx.build_jk_multi_dev(bad, dD.data_ptr(), dJ.data_ptr(), dK.data_ptr(), s)
    with pytest.raises(hfx.HfxError):
        ctx.build_jk_multi_dev(2, dD.data_ptr(), 0, 0, s)


def test_sp_shells_graphene_against_oracle():
    """SP (L) shells through the C ABI (written out as s and p on load): an
    8-carbon graphene bilayer's Fock matrix against the oracle's, the
    0.5 nm bilayer of the paper's table (44 carbons, 660 functions) on
    sampled shell blocks, and the 8-carbon SCF energy against the oracle's
    converged energy (fixture written by tests/golden/make_graphene_golden.py)."""
    import json
    import os
    import torch
    import oracle
    hfx = _hfx()
    m = W.graphene_bilayer(4)
    B = oracle.Basis(m)
    ctx = hfx.Context().load(m)
    assert ctx.nbf == 120 and ctx.nshell == 48
    D = W.random_symmetric(m.nbf, 14, 0.1)
    F, st = ctx.build_fock(D)
    ref, _, _ = _fock_ref(B, D)
    _, _, ost = B.jk(D, 1e-10)
    assert st.quartets_fp64 == ost[0]
    assert np.abs(F - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "graphene8_oracle_scf.json")))
    assert g["converged"]
    r = ctx.scf(e_tol=g["e_tol"], d_rms_tol=g["d_rms_tol"], max_iter=200)
    assert r["converged"]
    assert abs(r["energy"] - g["energy"]) < 1e-8, (r["energy"], g["energy"])
    m5 = W.graphene_bilayer(W.GRAPHENE_SIZES["0.5nm"])
    c5 = hfx.Context().load(m5)
    assert c5.nbf == 660
    D5 = W.random_orthonormal_density(m5.nbf, m5.nocc, 15)
    dD = torch.tensor(D5, device="cuda")
    J, K = torch.empty_like(dD), torch.empty_like(dD)
    s = torch.cuda.current_stream().cuda_stream
    c5.build_2e_dev(dD.data_ptr(), 1.0, 0.0, J.data_ptr(), s)
    c5.build_2e_dev(dD.data_ptr(), 0.0, -1.0, K.data_ptr(), s)
    torch.cuda.synchronize()
    J, K = J.cpu().numpy(), K.cpu().numpy()
    B5 = oracle.Basis(m5)
    bf = B5.shell_bf
    for a, b in [(0, 0), (1, 2), (2, 5), (3, 130), (262, 7)]:
        Jb, Kb = B5.jk_block(a, b, D5, 1e-10)
        na, nb = Jb.shape
        assert np.abs(J[bf[a]:bf[a] + na, bf[b]:bf[b] + nb] - Jb).max() < 1e-10, (a, b)
        assert np.abs(K[bf[a]:bf[a] + na, bf[b]:bf[b] + nb] - Kb).max() < 1e-10, (a, b)
